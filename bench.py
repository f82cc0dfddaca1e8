#!/usr/bin/env python
"""Throughput of the photon-guiding hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input:
  splat_histograms -> reconstruct_density (normalise + network)
  -> build_cdf -> sample_dirs -> eval_pdf (of the sampled directions)
and, for the clustered workload, build_hierarchy first.

Default workload: the clustered photons -- 5e7 photons in 64 Gaussian
clusters, an octree split while a voxel holds more than 8192 photons (depth
<= 6, 18,595 leaves), 128x128 maps, the 4-level U-Net (16/32/64/128) in FP32
mode (FP32 weights, FP64 activations and accumulation), 1e8 guided samples;
the hierarchy is built inside every step. After it, the uniform batch (1024
leaves x 4096 photons, 64x64 maps, 1,048,576 samples, leaf grouping given)
is timed the same way and reported under "uniform_batch".

Prints one JSON line (rank 0): leaves reconstructed per second over whole
steps, guided samples per second of the sampling stage, p50/p99 step
latency, the roofline of the dominant stage, and the FP64 CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import struct
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "fp64_mfma_TFLOPs": 78.6,
    "fp32_mfma_TFLOPs": 157.3,
    "bf16_mfma_TFLOPs": 2500.0,
    "fp8_mfma_TFLOPs": 5000.0,
}


def _model_shapes(model: bytes):
    arch, levels, n = struct.unpack_from("<III", model, 8)
    off = 20
    shapes = []
    for _ in range(n):
        co, ci, k = struct.unpack_from("<III", model, off)
        shapes.append((co, ci, k))
        off += 12 + 4 * (co * ci * k * k + co)
    return arch, levels, shapes


def _paper_schedule(shapes, D: int, px: int):
    """The paper-style U-Net's convs in execution order: (cout, cin, k,
    output pixels, kind) with kind 'first', 'pool' (2x2-pooled input),
    'res' (residual link), 'cat' (upsampled + skip input) or 'head'."""
    out, li = [], 0
    for d in range(D):
        p = px >> (2 * d)
        for j in range(3 if d == D - 1 else 2):
            co, ci, k = shapes[li + j]
            out.append((co, ci, k, p, "res" if j else ("first" if d == 0 else "pool")))
        li += 3 if d == D - 1 else 2
    for d in range(D - 2, -1, -1):
        p = px >> (2 * d)
        for j in range(2):
            co, ci, k = shapes[li + j]
            out.append((co, ci, k, p, "res" if j else "cat"))
        li += 2
    co, ci, k = shapes[li]
    out.append((co, ci, k, px, "head"))
    return out


def model_flops_per_leaf(model: bytes, H: int, W: int) -> float:
    """Algorithmic FLOPs of one leaf: 2*Cin*Cout*k*k per output pixel and
    layer, at each layer's resolution (pool/upsample/activations and
    residual adds not counted)."""
    arch, levels, shapes = _model_shapes(model)
    px = H * W
    if arch == 3:
        return float(sum(2 * ci * co * k * k * p for co, ci, k, p, _ in _paper_schedule(shapes, levels, px)))
    if arch == 1:
        return float(sum(2 * ci * co * k * k * px for co, ci, k in shapes))
    D = levels
    tot = 0.0
    for d in range(D):
        p = px >> (2 * d)
        for co, ci, k in shapes[2 * d:2 * d + 2]:
            tot += 2 * ci * co * k * k * p
    li = 2 * D
    for d in range(D - 2, -1, -1):
        p = px >> (2 * d)
        for co, ci, k in shapes[li:li + 2]:
            tot += 2 * ci * co * k * k * p
        li += 2
    co, ci, k = shapes[li]
    tot += 2 * ci * co * k * k * px
    return tot


def phase_saved_flops_per_leaf(model: bytes, H: int, W: int) -> float:
    """FLOPs that the FP32-mode decoder convolutions do not issue: on their
    nearest-upsampled channels (as many as the previous conv's outputs) a
    3x3 conv takes 4 phase-merged taps per output pixel instead of 9."""
    arch, levels, shapes = _model_shapes(model)
    px = H * W
    if arch == 1:
        return 0.0
    if arch == 3:
        sched = _paper_schedule(shapes, levels, px)
        return float(sum(2 * sched[i - 1][0] * co * 5 * p
                         for i, (co, ci, k, p, kind) in enumerate(sched) if kind == "cat"))
    saved, li = 0.0, 2 * levels
    for d in range(levels - 2, -1, -1):
        saved += 2 * shapes[li - 1][0] * shapes[li][0] * 5 * (px >> (2 * d))
        li += 2
    return saved


def model_bytes_per_leaf(model: bytes, H: int, W: int, esz: int, in_bytes: float = 8.0) -> float:
    """Algorithmic HBM bytes of one leaf's network pass: every layer reads its
    input once (in_bytes per pixel for the first layer: the u64 energy map,
    or u64 + u32 maps of two iterations for the five-channel input; pooled
    and concatenated inputs at their stored resolution) and writes its output
    once (esz bytes per activation, float32 densities for the last layer);
    a residual link reads its tensor once more."""
    arch, levels, shapes = _model_shapes(model)
    n = len(shapes)
    px = H * W
    if arch == 3:
        b, prev = 0.0, None                        # prev: (channels, pixels) of the last output
        skips = {}
        sched = _paper_schedule(shapes, levels, px)
        for i, (co, ci, k, p, kind) in enumerate(sched):
            if kind == "first":
                b += in_bytes * p
            elif kind == "pool":
                b += prev[0] * prev[1] * esz       # the pooled input read at full size
            elif kind == "res":
                b += 2 * prev[0] * prev[1] * esz   # input and residual
            elif kind == "cat":
                b += prev[0] * prev[1] * esz + skips[p] * p * esz
            else:                                  # head
                b += prev[0] * prev[1] * esz + 4 * p
                break
            b += co * p * esz
            prev = (co, p)
            nxt = sched[i + 1][4] if i + 1 < len(sched) else None
            if kind == "res" and nxt == "pool":
                skips[p] = co                      # an encoder level's output is its skip
        return b
    if arch == 1:
        b = in_bytes * px
        for i, (co, ci, k) in enumerate(shapes):
            if i:
                b += ci * px * esz
            b += (4 if i == n - 1 else co * esz) * px
        return b
    D = levels
    b = in_bytes * px                              # input maps
    out = []                                       # (channels, pixels) of each layer's output
    for d in range(D):
        p = px >> (2 * d)
        for j, (co, ci, k) in enumerate(shapes[2 * d:2 * d + 2]):
            if d or j:
                src_c, src_p = out[-1]
                b += src_c * src_p * esz           # previous output (pooled inputs read at full size)
            out.append((co, p))
            b += co * p * esz
    li = 2 * D
    for d in range(D - 2, -1, -1):
        p = px >> (2 * d)
        lo_c, lo_p = out[-1]
        skip_c, skip_p = out[2 * d + 1]
        co, ci, k = shapes[li]
        b += lo_c * lo_p * esz + skip_c * skip_p * esz + co * p * esz
        out.append((co, p))
        co2, ci2, k2 = shapes[li + 1]
        b += co * p * esz
        if d == 0:
            b += 4 * p                             # fused 1x1 head: float32 densities
        else:
            b += co2 * p * esz
            out.append((co2, p))
        li += 2
    return b


def sha_of(*paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pdf_errors_vs_fp32(npg, ctx, model, energy, precision, maps5=None):
    """Per-leaf L1 and KL of the low-precision pdf against the FP32 path's
    (which matches the FP64 oracle within 1e-5 relative), over every leaf.
    maps5: (count, energy_prev, count_prev) of a five-channel model."""
    import torch
    if maps5 is None:
        run = lambda p: npg.reconstruct_density(ctx, model, energy, p).double()
    else:
        run = lambda p: npg.reconstruct_density5(ctx, model, energy, *maps5, p).double()
    lo = run(precision)
    hi = run("fp32")
    L = lo.shape[0]
    p = lo.reshape(L, -1)
    q = hi.reshape(L, -1)
    p = p / p.sum(1, keepdim=True)
    q = q / q.sum(1, keepdim=True)
    l1 = (p - q).abs().sum(1)
    kl = torch.where(q > 0, q * torch.log(q / p.clamp_min(1e-300)), torch.zeros_like(q)).sum(1)
    qs = lambda t, f: float(torch.quantile(t.float(), f)) if t.numel() > 1 else float(t[0])
    return {"leaves": L, "l1_median": qs(l1, 0.5), "l1_p99": qs(l1, 0.99), "l1_max": float(l1.max()),
            "kl_median": qs(kl, 0.5), "kl_p99": qs(kl, 0.99), "kl_max": float(kl.max())}


def sampling_chi2(npg, ctx, tabs, L, H, W, n_leaves=64, per=100_000, seed=4343):
    """Chi-square tests of guided samples against the tables they were drawn
    from: n_leaves leaves evenly spread over the batch, `per` samples each;
    bins are merged in ascending expectation until each group expects >= 5.
    Returns the spread of the per-leaf p-values and a KS test of their
    uniformity (a correct sampler gives uniform p-values)."""
    import torch
    from scipy import stats
    dev = tabs.pdf.device
    leaves = np.unique(np.linspace(0, L - 1, min(n_leaves, L)).astype(np.int64))
    q_leaf = torch.from_numpy(np.repeat(leaves, per).astype(np.int32)).to(dev)
    g = torch.Generator(device=dev).manual_seed(seed)
    u = torch.rand((q_leaf.shape[0], 2), generator=g, device=dev)
    _, _, b = npg.sample_dirs(ctx, tabs, q_leaf, u)
    b = b.cpu().numpy().view(np.uint32).astype(np.int64).reshape(len(leaves), per)
    pdf = tabs.pdf[torch.from_numpy(leaves).to(dev)].double().cpu().numpy().reshape(len(leaves), -1)
    pv = []
    for k in range(len(leaves)):
        pk = pdf[k] / pdf[k].sum()
        obs = np.bincount(b[k], minlength=H * W).astype(np.float64)
        exp = pk * per
        order = np.argsort(exp)
        o_m, e_m, oc, ec = [], [], 0.0, 0.0
        for j in order:
            if exp[j] == 0:
                continue
            oc += obs[j]
            ec += exp[j]
            if ec >= 5:
                o_m.append(oc)
                e_m.append(ec)
                oc = ec = 0.0
        if ec > 0 and o_m:
            o_m[-1] += oc
            e_m[-1] += ec
        o_m, e_m = np.array(o_m), np.array(e_m)
        chi = float(((o_m - e_m) ** 2 / e_m).sum())
        pv.append(float(stats.chi2.sf(chi, len(o_m) - 1)))
    pv = np.array(pv)
    return {"leaves": int(len(leaves)), "samples_per_leaf": per, "pvalue_min": float(pv.min()),
            "pvalue_median": float(np.median(pv)), "frac_below_0.01": float((pv < 0.01).mean()),
            "ks_uniform_p": float(stats.kstest(pv, "uniform").pvalue)}


def _omp(threads: int | None = None) -> int:
    """Sets (if given) and returns the OpenMP thread count of the oracle
    library's runtime (libgomp, loaded with it)."""
    import ctypes as C
    gomp = C.CDLL("libgomp.so.1")
    if threads is not None:
        gomp.omp_set_num_threads(int(threads))
    return int(gomp.omp_get_max_threads())


def host_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "os_cpu_count": os.cpu_count()}


def _oracle_chain(orc, b_dirs, b_w, leaf_off, H, W, model, n_queries, seed, perm=None, input5=None, times=None):
    """The oracle's whole step on a set of leaves: splat -> normalise ->
    network -> CDF -> n_queries guided samples -> pdf of the sampled
    directions; `times` (a dict) collects the seconds of each stage."""
    from paper_2010_01775_amd import synth
    t = {} if times is None else times
    mark = [time.perf_counter()]

    def lap(stage):
        now = time.perf_counter()
        t[stage] = t.get(stage, 0.0) + now - mark[0]
        mark[0] = now

    rc, E, P = orc.splat(b_dirs, b_w, leaf_off, H, W, perm=perm)
    lap("splat")
    if input5 is None:
        x = orc.normalize_input(E)
        lap("normalise")
        rc, dens = orc.net_forward(model, x)
    else:
        Ep, Pp = input5
        x = orc.input5(E, Ep, P, Pp)
        lap("normalise")
        rc, dens = orc.net_forward5(model, x)
    assert rc == 0
    lap("network")
    rc, pdf, marg, cond, total = orc.build_cdf(dens)
    assert rc == 0
    lap("cdf")
    ql, qu = synth.queries(seed, pdf.shape[0], n_queries)
    mark[0] = time.perf_counter()   # query generation is not the oracle's work
    rc, d, p, bins = orc.sample(pdf, marg, cond, ql, qu)
    lap("sample")
    rc, pe = orc.eval_pdf(pdf, ql, d.astype(np.float32))
    lap("eval")
    return pdf


def cpu_baseline_uniform(input5: bool = False, model5: bytes | None = None):
    """The FP64 oracle, as it stands, on a bounded sample of the uniform batch
    (about 15 s of CPU work on 16 cores)."""
    from oracle import oracle as orc
    from paper_2010_01775_amd import synth

    threads = _omp()
    L = max(16, threads * 120)
    b = synth.uniform_batch(L=L, n_queries=L * 1024)
    prev = None
    model = b.model
    if input5:
        # iteration t-1 = first half of each leaf's photons, as in the GPU run
        off = b.leaf_off.astype(np.int64)
        half = (off[1:] - off[:-1]) // 2
        perm_p = np.concatenate([np.arange(off[l], off[l] + half[l]) for l in range(L)]).astype(np.uint32)
        off_p = np.concatenate([[0], np.cumsum(half)]).astype(np.uint32)
        model = model5 or synth.unet5_model(1003)
        rc, Ep, Pp = orc.splat(b.dirs, b.w, off_p, b.H, b.W, perm=perm_p)   # resident, not timed
        prev = (Ep, Pp)
    stages = {}
    _oracle_chain(orc, b.dirs, b.w, b.leaf_off, b.H, b.W, model, L * 1024, 77, input5=prev, times=stages)
    dt = sum(stages.values())
    return {"value": L / dt, "unit": "leaves/s", "cores": min(threads, L), "kind": "oracle",
            "sample": f"{L} leaves x 4096 photons (64x64, {'five-channel ' if input5 else ''}network, FP64) "
                      f"end to end plus {L * 1024} samples and their pdfs; {dt:.1f} s",
            "stage_s_per_step": {k: v * 1024 / L for k, v in stages.items()},
            "host": host_info()}


def cpu_baseline_clustered(cp, model: bytes, L_gpu: int, n_queries: int, subset: int = 512,
                           subset_1t: int = 16):
    """The FP64 oracle, as it stands, on the clustered workload: its octree
    over all photons (timed whole), then the rest of the step on `subset`
    leaves stratified by photon count (every L/subset-th leaf in count order,
    so the subset's photons per leaf follow the workload's distribution) with
    the queries scaled by subset/L; extrapolated to the whole step as
    t_tree + t_subset * L/subset.  The same with one thread (tree timed whole,
    the chain on `subset_1t` stratified leaves)."""
    from oracle import oracle as orc

    def run(n_sub):
        t0 = time.perf_counter()
        rc, tree = orc.build_tree(cp.pos, 8192, 6, max_leaves=1 << 20)
        t_tree = time.perf_counter() - t0
        assert rc == 0
        L = tree["n_leaves"]
        off = tree["leaf_off"].astype(np.int64)
        cnt = np.diff(off)
        pick = stratified_leaves(cnt, n_sub)
        sub_perm = np.concatenate([tree["perm"][off[l]:off[l + 1]] for l in pick])
        sub_off = np.concatenate([[0], np.cumsum(cnt[pick])]).astype(np.uint32)
        nq = max(1, int(round(n_queries * n_sub / L)))
        stages = {}
        _oracle_chain(orc, cp.dirs, cp.w, sub_off, 128, 128, model, nq, 78, perm=sub_perm, times=stages)
        t_sub = sum(stages.values())
        t_full = t_tree + t_sub * L / n_sub
        per_step = {"hierarchy": t_tree} | {k: v * L / n_sub for k, v in stages.items()}
        return L, int(cnt[pick].sum()), nq, t_tree, t_sub, t_full, per_step

    threads = _omp()
    L, ph, nq, t_tree, t_sub, t_full, per_step = run(subset)
    if L != L_gpu:
        raise RuntimeError(f"oracle tree has {L} leaves, the GPU's {L_gpu}")
    _omp(1)
    try:
        _, ph1, nq1, t_tree1, t_sub1, t_full1, _ = run(subset_1t)
    finally:
        _omp(threads)
    return {"value": L / t_full, "unit": "leaves/s", "cores": threads, "kind": "oracle",
            "sample": (f"octree over all 5e7 photons ({t_tree:.1f} s), then splat/normalise/network/CDF/"
                       f"{nq} samples + pdfs on {subset} leaves stratified by photon count ({ph} photons, "
                       f"128x128, FP64; {t_sub:.1f} s); extrapolated to all {L} leaves and 1e8 samples as "
                       f"t_tree + t_subset * {L}/{subset} = {t_full:.1f} s per step"),
            "subset_leaves_per_s": subset / t_sub,
            "stage_s_per_step": per_step,
            "one_thread": {"value": L / t_full1, "unit": "leaves/s", "cores": 1,
                           "sample": f"octree ({t_tree1:.1f} s) + {subset_1t} stratified leaves "
                                     f"({ph1} photons, {nq1} samples; {t_sub1:.1f} s), extrapolated "
                                     f"to {t_full1:.0f} s per step"},
            "host": host_info()}


def run_serving(args):
    """The serving stream: Poisson arrivals of reconstruction requests (1-4096
    leaves, lognormal photons per leaf in [256, 1e6], 64x64 or 128x128) and
    sampling batches (1e4-1e7 queries on resident leaves), interleaved 1:1.
    The arrival rate is set so that FP32 processing one request at a time
    would be ~70 % busy.  The same stream runs through the server twice: BF16
    with continuous batching on 4 slots, and FP32 one request at a time."""
    import torch

    from paper_2010_01775_amd import npg, synth

    dev = "cuda:0"
    ctx = npg.Context(0)
    model = npg.Model(ctx, synth.unet_model(1004))
    pool = synth.uniform_batch(seed=1004, L=4096, per_leaf=4096, H=64, W=64, n_queries=1, model=b"")
    n_pool = pool.dirs.shape[0]
    dirs = torch.from_numpy(pool.dirs).to(dev)
    w = torch.from_numpy(pool.w.view(np.int32)).to(dev)
    qmax = 10_000_000
    u = torch.from_numpy(np.stack([synth.uniforms(synth.rng_for(5), qmax), synth.uniforms(synth.rng_for(6), qmax)],
                                  1)).to(dev)
    outs = [(torch.empty((qmax, 3), device=dev), torch.empty(qmax, device=dev)) for _ in range(4)]
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)

    def windows(req, seed):
        rng = np.random.default_rng(seed)
        cnt = req.counts.astype(np.uint32)
        beg = (rng.random(len(cnt)) * (n_pool - cnt)).astype(np.uint32)
        return beg, cnt

    def run(stream, prec, n_slots, max_batch, paced=True):
        srv = npg.Server(ctx, model, n_slots=n_slots, max_batch_leaves=max_batch, table_bytes=48 << 30,
                         slot_scratch_bytes=3 << 30, precision=prec)
        resident, tickets, kinds, leaves, queries = [], [], [], 0, 0
        lat_of = {}  # latency of released reconstructions (their tickets are gone after release)
        gs = torch.cuda.Stream()
        t0 = time.perf_counter()
        for i, req in enumerate(stream):
            if paced:
                while time.perf_counter() - t0 < req.t_arrive:
                    time.sleep(0.0002)
            if req.kind == "recon":
                beg, cnt = windows(req, req.seed)
                t = srv.submit_recon(dirs, w, beg, cnt, req.H, req.W)
                resident.append((t, req.n_leaves))
                if len(resident) > 64:
                    old = resident.pop(0)[0]
                    lat_of[old] = srv.wait(old)
                    srv.release(old)
                tickets.append(t)
                kinds.append(("recon", req.n_leaves))
                leaves += req.n_leaves
            else:
                if not resident:
                    continue
                tr, L = resident[int(np.random.default_rng(req.seed).integers(0, len(resident)))]
                n = min(req.n_queries, qmax)
                with torch.cuda.stream(gs):
                    leaf = torch.randint(0, L, (n,), device=dev, dtype=torch.int32, generator=gen)
                gs.synchronize()
                d, p = outs[i % 4]
                tickets.append(srv.submit_sample(tr, leaf, u[:n], d, p))
                kinds.append(("sample", n))
                queries += n
        lat = [lat_of[t] if t in lat_of else srv.wait(t) for t in tickets]
        t_end = time.perf_counter()
        st = srv.stats()
        srv.close()
        lat_r = [l for l, k in zip(lat, kinds) if k[0] == "recon"]
        lat_s = [l for l, k in zip(lat, kinds) if k[0] == "sample"]
        span = t_end - t0
        return {"leaves_per_s": leaves / span, "samples_per_s": queries / span, "seconds": span,
                "p50_ms": float(np.percentile(lat, 50)) / 1e3, "p99_ms": float(np.percentile(lat, 99)) / 1e3,
                "recon_p50_ms": float(np.percentile(lat_r, 50)) / 1e3,
                "recon_p99_ms": float(np.percentile(lat_r, 99)) / 1e3,
                "sample_p50_ms": float(np.percentile(lat_s, 50)) / 1e3 if lat_s else None,
                "sample_p99_ms": float(np.percentile(lat_s, 99)) / 1e3 if lat_s else None,
                "batches": st["batches"], "merged_requests": st["merged_requests"],
                "max_concurrent": st["max_concurrent"], "requests": len(tickets)}

    # service time of the FP32 one-at-a-time form, to set the arrival rate:
    # the whole stream back to back (arrival times scale with 1/rate, the
    # requests themselves do not depend on it)
    unpaced = run(synth.serving_stream(seed=1004, n_requests=args.requests, rate_hz=1e9), "fp32", 1, 0,
                  paced=False)
    mean_service = unpaced["seconds"] / unpaced["requests"]
    rate = 0.7 / mean_service
    stream = synth.serving_stream(seed=1004, n_requests=args.requests, rate_hz=rate)
    print(f"serving: mean FP32 service {mean_service * 1e3:.2f} ms -> rate {rate:.1f} req/s", file=sys.stderr,
          flush=True)
    # saturation: the same requests back to back through the served form
    sat = run(synth.serving_stream(seed=1004, n_requests=args.requests, rate_hz=1e9), "bf16", 4, 8192, paced=False)
    print(f"served bf16 saturated: {sat}", file=sys.stderr, flush=True)
    served = run(stream, "bf16", 4, 8192)
    print(f"served bf16: {served}", file=sys.stderr, flush=True)
    base = run(stream, "fp32", 1, 0)
    print(f"fp32 unbatched: {base}", file=sys.stderr, flush=True)
    res = {
        "metric": "leaf densities reconstructed/sec + guided samples/sec; p50/p99 batch latency",
        "value": sat["leaves_per_s"], "unit": "leaves/s", "n_gpus": 1, "steps": args.requests,
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 conv, f32 accumulation (served); baseline f32 weights, f64 activations and accumulation",
        "data": "synthetic (seeded vMF-mixture photon pool, lognormal leaf sizes, Poisson arrivals)",
        "config": {"workload": f"serving stream: {args.requests} requests, Poisson {rate:.1f}/s "
                               f"(FP32 one-at-a-time ~70% busy), recon 1-4096 leaves x 256-1e6 photons at 64^2/"
                               f"128^2, sampling 1e4-1e7 queries, 1:1", "rate_hz": rate,
                   "mean_fp32_service_ms": mean_service * 1e3},
        "saturated": {"served_bf16": sat, "fp32_unbatched": unpaced,
                      "note": "requests submitted back to back; value = served leaves/s"},
        "at_70pct_of_fp32_capacity": {"served_bf16": served, "fp32_unbatched": base},
        "p50_ms": served["p50_ms"], "p99_ms": served["p99_ms"], "samples_per_s": sat["samples_per_s"],
    }
    print(json.dumps(res))
    model.free()
    ctx.close()


def stage_bytes(stage: str, n_photons: int, L: int, H: int, W: int, nq: int, sorted_photons: bool = False) -> float:
    """Algorithmic HBM bytes of one stage: what the step must read and write
    once (no sort passes, no re-reads).
      hier   positions 12 B read + permutation 4 B written per photon, leaf
             offsets 4 B per leaf (leaf_of is not requested by the step);
             with the photons put in leaf order (the octree) also their
             direction and weight, 16 B read and 16 B written per photon
      splat  direction 12 B + weight 4 B read per photon; energy 8 B + count
             4 B written per bin
      cdf    density 4 B read; pdf 4 B, conditional 4 (W+1)/W B written per
             bin; marginal 4 (H+1) B and total 8 B per leaf
      sample query 12 B read, direction 12 B + pdf 4 B + bin 4 B written;
             the tables (pdf, conditional, marginal) read once
      eval   leaf 4 B + direction 12 B read, pdf 4 B written per query; the
             pdf table read once"""
    bins = float(L) * H * W
    tab = bins * 4 + L * H * (W + 1) * 4.0 + L * (H + 1) * 4.0
    return {"hier": n_photons * (48.0 if sorted_photons else 16.0) + (L + 1) * 4.0,
            "splat": n_photons * 16.0 + bins * 12.0,
            "cdf": bins * 4.0 + tab + L * 8.0,
            "sample": nq * 32.0 + tab,
            "eval": nq * 20.0 + bins * 4.0}[stage]


def stratified_leaves(counts: np.ndarray, n: int) -> np.ndarray:
    """n leaves spread evenly over the photon-count order (sorted ids)."""
    order = np.argsort(counts, kind="stable")
    return np.sort(order[np.linspace(0, len(counts) - 1, min(n, len(counts))).astype(np.int64)])


def fp8_calibration_maps(npg, ctx, workload: str, H: int, W: int):
    """Energy maps of the FP8 calibration set: 256 leaves of the same
    workload drawn from seed + 100 (the uniform batch: seed 1101; the
    clustered workload: seed 1103, its own octree, leaves stratified by
    photon count).  Returns (maps on cuda:0, description)."""
    import torch

    from paper_2010_01775_amd import synth
    dev = "cuda:0"
    i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    if workload == "uniform":
        cb = synth.uniform_batch(seed=1101, L=256, n_queries=1, model=b"")
        ce, _ = npg.splat_histograms(ctx, f32(cb.dirs), i32(cb.w), i32(cb.leaf_off), H, W, want_count=False)
        return ce, "256 leaves of the uniform batch drawn from seed 1101"
    ccp = synth.clustered_photons(seed=1103)
    chier = npg.build_hierarchy(ctx, f32(ccp.pos), 8192, 6, max_leaves=65536)
    coff = chier["leaf_off"].cpu().numpy().view(np.uint32).astype(np.int64)
    cperm = chier["perm"].cpu().numpy().view(np.uint32)
    pick = stratified_leaves(np.diff(coff), 256)
    sel = np.concatenate([cperm[coff[l]:coff[l + 1]] for l in pick])
    soff = np.concatenate([[0], np.cumsum(np.diff(coff)[pick])]).astype(np.uint32)
    ce, _ = npg.splat_histograms(ctx, f32(ccp.dirs[sel]), i32(ccp.w[sel]), i32(soff), H, W, want_count=False)
    return ce, (f"256 leaves stratified by photon count from the clustered workload drawn from seed 1103 "
                f"(its own octree, {chier['n_leaves']} leaves)")


def run_path(args, workload: str, with_baseline: bool = True) -> dict:
    """Times `args.steps` steps of the hot path on one workload; returns the
    JSON record."""
    import torch

    from paper_2010_01775_amd import npg, synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

    ctx = npg.Context(0)
    cp = None
    if workload == "uniform":
        b = synth.uniform_batch()
        H, W, L = b.H, b.W, b.L
        dirs, w, off = f32(b.dirs), i32(b.w), i32(b.leaf_off)
        q_leaf, q_u = i32(b.q_leaf), f32(b.q_u)
        model_bytes = b.model
        pos = None
        n_photons = b.dirs.shape[0]
        desc = ("uniform batch: 1024 leaves x 4096 photons (vMF mixtures), 64x64 equal-area maps, "
                "U-Net 16/32/64/128, 1048576 guided samples")
    else:
        cp = synth.clustered_photons()
        n_photons = cp.pos.shape[0]
        # the paper's grid yields ~20x more (and smaller) leaves than the
        # octree: 64x64 maps keep their tables within HBM
        H = W = 64 if args.hierarchy == "kdgrid" else 128
        pos, dirs, w = f32(cp.pos), f32(cp.dirs), i32(cp.w)
        model_bytes = synth.unet_model(1002)
        if args.hierarchy == "kdgrid":
            kprm = npg.kdgrid_params()
            knrm = f32(synth.surface_normals(1003, cp.pos))
            kvalid = npg.mark_valid(ctx, kprm, f32(synth.bounce_points(1004, cp.pos, 2_000_000)))
            out = npg.build_kdgrid(ctx, kprm, pos, knrm, kvalid, max_leaves=1 << 20)
            hier_desc = (f"paper hierarchy: 100^3 grid, valid voxels from 2e6 bounce points, local KD split "
                         f"count > {kprm.split_count:.1f} or normal variance > 0.5, depth <= 8")
        else:
            out = npg.build_hierarchy(ctx, pos, 8192, 6, max_leaves=65536)
            hier_desc = "octree split > 8192 depth <= 6"
        L = out["n_leaves"]
        ql, qu = synth.queries(1102, L, 100_000_000)
        q_leaf, q_u = i32(ql), f32(qu)
        del ql, qu
        desc = (f"clustered: 5e7 photons in 64 Gaussian clusters, {hier_desc} "
                f"({L} leaves), {H}x{W} maps, U-Net 16/32/64/128, 1e8 guided samples")
    if args.input5:
        model_bytes = synth.paper_unet_model(1006) if args.paper_net else synth.unet5_model(1003)
    model = npg.Model(ctx, model_bytes)
    experts = [model] + [npg.Model(ctx, synth.unet_model(2000 + k)) for k in range(4)] if args.experts else None
    nq = q_leaf.shape[0]
    flops_leaf = model_flops_per_leaf(model_bytes, H, W)

    # preallocated outputs
    energy = torch.empty((L, H, W), dtype=torch.int64, device=dev)
    count = torch.empty((L, H, W), dtype=torch.int32, device=dev)
    dens = torch.empty((L, H, W), dtype=torch.float32, device=dev)
    tabs = npg.CdfTables(torch.empty((L, H, W), dtype=torch.float32, device=dev),
                         torch.empty((L, H + 1), dtype=torch.float32, device=dev),
                         torch.empty((L, H, W + 1), dtype=torch.float32, device=dev),
                         torch.empty(L, dtype=torch.float64, device=dev))
    sd = (torch.empty((nq, 3), dtype=torch.float32, device=dev),
          torch.empty(nq, dtype=torch.float32, device=dev),
          torch.empty(nq, dtype=torch.int32, device=dev))
    pe = torch.empty(nq, dtype=torch.float32, device=dev)
    prev = None
    if args.input5:
        # maps of iteration t-1, resident before timing: the first half of each
        # leaf's photons (photon maps accumulate over iterations)
        lo_ = out["leaf_off"][:L + 1].long() if pos is not None else off[:L + 1].long()
        half = (lo_[1:] - lo_[:-1]) // 2
        off_p = torch.zeros(L + 1, dtype=torch.int64, device=dev)
        off_p[1:] = torch.cumsum(half, 0)
        leaf_id = torch.repeat_interleave(torch.arange(L, device=dev), half)
        idx = lo_[leaf_id] + torch.arange(leaf_id.shape[0], device=dev) - off_p[leaf_id]
        perm_p = (out["perm"].long()[idx] if pos is not None else idx).to(torch.int32)
        prev = (torch.empty((L, H, W), dtype=torch.int64, device=dev),
                torch.empty((L, H, W), dtype=torch.int32, device=dev))
        npg.splat_histograms(ctx, dirs, w, off_p.to(torch.int32), H, W, perm=perm_p, energy=prev[0], count=prev[1])
        del leaf_id, idx, perm_p
    hier_out = None
    if pos is not None:
        n = pos.shape[0]
        cap = (1 << 20) if args.hierarchy == "kdgrid" else 65536
        hier_out = dict(perm=torch.empty(n, dtype=torch.int32, device=dev),
                        off=torch.empty(cap + 1, dtype=torch.int32, device=dev))
        if args.hierarchy == "octree":
            # the photons in leaf order, written by the build
            hier_out["dirs"] = torch.empty((n, 3), dtype=torch.float32, device=dev)
            hier_out["w"] = torch.empty(n, dtype=torch.int32, device=dev)
        if args.hierarchy == "kdgrid":
            hier_out["root"] = torch.empty(100 ** 3, dtype=torch.int32, device=dev)
            hier_out["nodes"] = torch.empty((2 * cap, 2), dtype=torch.int32, device=dev)

    stages = ["hier", "splat", "recon", "cdf", "sample", "eval"] if pos is not None else \
             ["splat", "recon", "cdf", "sample", "eval"]
    ev = {s: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for s in stages}
    stream = torch.cuda.current_stream()

    expert_leaves = [0] * 5

    def step(record):
        def mark(s, i):
            if record:
                ev[s][i].record(stream)
        if pos is not None:
            import ctypes as C
            mark("hier", 0)
            nl = C.c_uint32(0)
            if args.hierarchy == "kdgrid":
                nn = C.c_uint32(0)
                ctx.check(ctx.lib.npg_build_kdgrid(ctx.h, C.byref(kprm), pos.data_ptr(), knrm.data_ptr(),
                                                   pos.shape[0], kvalid.data_ptr(), hier_out["perm"].data_ptr(),
                                                   hier_out["off"].data_ptr(), hier_out["root"].data_ptr(),
                                                   hier_out["nodes"].data_ptr(), 1 << 20, C.byref(nl),
                                                   C.byref(nn), stream.cuda_stream))
            else:
                prm = npg.HierParams(8192, 6)
                ctx.check(ctx.lib.npg_build_hierarchy_sorted(ctx.h, pos.data_ptr(), dirs.data_ptr(), w.data_ptr(),
                                                             pos.shape[0], C.byref(prm),
                                                             hier_out["perm"].data_ptr(),
                                                             hier_out["dirs"].data_ptr(), hier_out["w"].data_ptr(),
                                                             hier_out["off"].data_ptr(), None, None, 65536,
                                                             C.byref(nl), stream.cuda_stream))
            assert nl.value == L
            mark("hier", 1)
            lo = hier_out["off"][:L + 1]
            mark("splat", 0)
            if args.hierarchy == "octree":   # leaf-ordered photons: contiguous runs per leaf
                npg.splat_histograms(ctx, hier_out["dirs"], hier_out["w"], lo, H, W, energy=energy, count=count)
            else:
                npg.splat_histograms(ctx, dirs, w, lo, H, W, perm=hier_out["perm"], energy=energy, count=count)
        else:
            mark("splat", 0)
            npg.splat_histograms(ctx, dirs, w, off, H, W, energy=energy, count=count)
        mark("splat", 1)
        mark("recon", 0)
        if experts:
            lo = hier_out["off"][:L + 1] if pos is not None else off
            _, expert_leaves[:] = npg.reconstruct_experts(ctx, experts, lo, energy, args.precision, density=dens)
        elif prev is not None:
            npg.reconstruct_density5(ctx, model, energy, count, prev[0], prev[1], args.precision, density=dens)
        else:
            npg.reconstruct_density(ctx, model, energy, args.precision, count=count, density=dens)
        mark("recon", 1)
        mark("cdf", 0)
        npg.build_cdf(ctx, dens, out=tabs)
        mark("cdf", 1)
        mark("sample", 0)
        npg.sample_dirs(ctx, tabs, q_leaf, q_u, out=sd)
        mark("sample", 1)
        mark("eval", 0)
        npg.eval_pdf(ctx, tabs, q_leaf, sd[0], out=pe)
        mark("eval", 1)

    calib = None
    if args.precision == "fp8":
        # static e4m3 scales from a separate calibration set of the same
        # workload, set once before timing
        ce, calib = fp8_calibration_maps(npg, ctx, workload, H, W)
        for m in experts or [model]:
            m.calibrate_fp8(ce)
        del ce
    tune = None
    if not args.no_autotune:
        # per-layer pixel tiles and leaf-chunk size, chosen once before timing
        for m in experts or [model]:
            tune = npg.autotune(ctx, m, H, W, args.precision, probe_leaves=min(L, 1024))
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    if npg.sync_status(ctx) != 0:
        raise RuntimeError("data-dependent error during warm-up")

    def mis_rates(reps=3):
        """One-sample MIS on the final tables (outside the timed steps): the
        guided queries' uniforms plus a fresh selection uniform, random unit
        normals for the cosine-lobe BSDF, per-leaf alpha from synthetic path
        statistics; samples/s and evaluations/s."""
        g = torch.Generator(device=dev).manual_seed(4242)
        normal = torch.randn((nq, 3), generator=g, device=dev)
        normal /= normal.norm(dim=1, keepdim=True)
        u3 = torch.cat([torch.rand((nq, 1), generator=g, device=dev), q_u.view(nq, 2)], 1).contiguous()
        nu_b = torch.rand(L, generator=g, device=dev) * 4
        nu_g = torch.rand(L, generator=g, device=dev) * 4
        qcount = (torch.rand((2, L), generator=g, device=dev) * 200).to(torch.int32)
        alpha = npg.mis_alpha(ctx, nu_b, nu_g, qcount[0].contiguous(), qcount[1].contiguous())
        outs = (torch.empty((nq, 3), dtype=torch.float32, device=dev), torch.empty(nq, dtype=torch.float32, device=dev),
                torch.empty(nq, dtype=torch.uint8, device=dev))
        pe_m = torch.empty(nq, dtype=torch.float32, device=dev)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        ts, te = [], []
        for r in range(reps + 1):
            e0.record(stream)
            npg.sample_mis(ctx, tabs, alpha, q_leaf, normal, u3, out=outs)
            e1.record(stream)
            npg.eval_pdf_mis(ctx, tabs, alpha, q_leaf, normal, outs[0], out=pe_m)
            e2.record(stream)
            torch.cuda.synchronize()
            if r:  # the first pass warms up
                ts.append(e0.elapsed_time(e1))
                te.append(e1.elapsed_time(e2))
        if npg.sync_status(ctx) != 0:
            raise RuntimeError("data-dependent error in the MIS calls")
        res_ = {"mis_samples_per_s": nq / (np.mean(ts) / 1e3), "mis_eval_per_s": nq / (np.mean(te) / 1e3),
                "bsdf_fraction": float(outs[2].float().mean()), "mean_alpha": float(alpha.mean())}
        del normal, u3, outs, pe_m
        return res_

    def grouped_rates(reps=3):
        """The same queries sorted by leaf (a stable sort outside the timed
        region), as a caller that groups its path vertices by leaf would
        issue them: sampling and evaluation rates on the final tables, and a
        check that every query's result equals its result in random order."""
        order = torch.sort(q_leaf, stable=True).indices
        gl, gu = q_leaf[order].contiguous(), q_u[order].contiguous()
        out = (torch.empty((nq, 3), dtype=torch.float32, device=dev), torch.empty(nq, dtype=torch.float32, device=dev))
        pe_g = torch.empty(nq, dtype=torch.float32, device=dev)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        ts, te = [], []
        for r in range(reps + 1):
            e0.record(stream)
            npg.sample_dirs(ctx, tabs, gl, gu, out=(out[0], out[1], None))
            e1.record(stream)
            npg.eval_pdf(ctx, tabs, gl, out[0], out=pe_g)
            e2.record(stream)
            torch.cuda.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1))
                te.append(e1.elapsed_time(e2))
        if npg.sync_status(ctx) != 0:
            raise RuntimeError("data-dependent error in grouped sampling")
        same = bool(torch.equal(out[0], sd[0][order]) and torch.equal(out[1], sd[1][order]))
        del order, gl, gu, out, pe_g
        return {"samples_per_s": nq / (np.mean(ts) / 1e3), "eval_per_s": nq / (np.mean(te) / 1e3),
                "sample_ms": float(np.mean(ts)), "same_results_as_random_order": same,
                "order": "queries stably sorted by leaf before timing"}

    per_step, stage_ms = [], {s: [] for s in stages}
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    s0 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ctx.conv_flops(reset=True)
    t_start.record(stream)
    for k in range(args.steps):
        s0.record(stream)
        step(True)
        torch.cuda.synchronize()
        per_step.append(s0.elapsed_time(ev["eval"][1]))
        for s in stages:
            stage_ms[s].append(ev[s][0].elapsed_time(ev[s][1]))
        print(f"{workload} step {k}: {per_step[-1]:.2f} ms", file=sys.stderr, flush=True)
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    if npg.sync_status(ctx) != 0:
        raise RuntimeError("data-dependent error during the timed steps")
    mat_flops, vec_flops = (f / args.steps for f in ctx.conv_flops(reset=True))

    avg = {s: float(np.mean(v)) for s, v in stage_ms.items()}

    def fused_form(steps):
        """The same step with the batched-leaf entry: hierarchy (leaf-ordered
        photons) -> reconstruct_fused (splat, normalisation, network and CDF
        per leaf chunk, replayed as a HIP graph from its third call) ->
        sampling -> evaluation, on a side stream; identical results."""
        import ctypes as C
        fs = torch.cuda.Stream()
        ctx.set_option("graphs", 1)
        fe = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for k in ("step", "recon")}

        def one(record):
            if pos is not None:
                nl = C.c_uint32(0)
                prm = npg.HierParams(8192, 6)
                ctx.check(ctx.lib.npg_build_hierarchy_sorted(ctx.h, pos.data_ptr(), dirs.data_ptr(), w.data_ptr(),
                                                             pos.shape[0], C.byref(prm), hier_out["perm"].data_ptr(),
                                                             hier_out["dirs"].data_ptr(), hier_out["w"].data_ptr(),
                                                             hier_out["off"].data_ptr(), None, None, 65536,
                                                             C.byref(nl), fs.cuda_stream))
                src = (hier_out["dirs"], hier_out["w"], hier_out["off"][:L + 1])
            else:
                src = (dirs, w, off)
            if record:
                fe["recon"][0].record(fs)
            npg.reconstruct_fused(ctx, model, *src, H, W, args.precision, out=tabs, stream=fs)
            if record:
                fe["recon"][1].record(fs)
            npg.sample_dirs(ctx, tabs, q_leaf, q_u, out=sd, stream=fs)
            npg.eval_pdf(ctx, tabs, q_leaf, sd[0], out=pe, stream=fs)

        for _ in range(3):   # eager, captured, first replay
            one(False)
        fs.synchronize()
        t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        rec_ms, step_ms = [], []
        t0e.record(fs)
        for _ in range(steps):
            fe["step"][0].record(fs)
            one(True)
            fe["step"][1].record(fs)
            fs.synchronize()
            rec_ms.append(fe["recon"][0].elapsed_time(fe["recon"][1]))
            step_ms.append(fe["step"][0].elapsed_time(fe["step"][1]))
        t1e.record(fs)
        fs.synchronize()
        ctx.set_option("graphs", 0)
        if npg.sync_status(ctx, stream=fs) != 0:
            raise RuntimeError("data-dependent error in the fused form")
        tot = t0e.elapsed_time(t1e)
        return {"value": L * steps / (tot / 1e3), "unit": "leaves/s", "ms_per_step": tot / steps,
                "p50_ms": float(np.percentile(step_ms, 50)), "p99_ms": float(np.percentile(step_ms, 99)),
                "reconstruct_fused_ms": float(np.mean(rec_ms)),
                "form": "build_hierarchy_sorted -> reconstruct_fused (HIP graph replay) -> sample_dirs -> eval_pdf"
                        if pos is not None else "reconstruct_fused (HIP graph replay) -> sample_dirs -> eval_pdf"}

    fused = None
    if not args.experts and not args.input5 and (pos is None or args.hierarchy == "octree"):
        fused = fused_form(max(3, args.steps // 2))
        print(f"{workload} fused form: {fused['ms_per_step']:.2f} ms per step", file=sys.stderr, flush=True)
    mis = mis_rates()
    grouped = grouped_rates()
    locate = None
    if pos is not None and args.hierarchy == "kdgrid":
        # point location at render time (outside the timed steps): 2e7 points
        # near where photons land, with the grid of the last timed build
        kq = f32(synth.bounce_points(1005, cp.pos, 20_000_000))
        grid = dict(cell_root=hier_out["root"], nodes=hier_out["nodes"], n_nodes=int(out["n_nodes"]))
        kl = torch.empty(kq.shape[0], dtype=torch.int32, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tl = []
        for r in range(4):
            e0.record(stream)
            npg.locate(ctx, kprm, grid, kq, out=kl)
            e1.record(stream)
            torch.cuda.synchronize()
            if r:
                tl.append(e0.elapsed_time(e1))
        if npg.sync_status(ctx) != 0:
            raise RuntimeError("data-dependent error in point location")
        locate = {"queries": kq.shape[0], "per_s": kq.shape[0] / (np.mean(tl) / 1e3),
                  "located_fraction": float((kl != -1).float().mean()),
                  "build_photons_per_s": pos.shape[0] / (avg["hier"] / 1e3), "nodes": int(out["n_nodes"])}
    recon_s = avg["recon"] / 1e3
    flops = flops_leaf * L
    if args.precision == "fp32":
        peak, peak_name = PEAK["fp64_mfma_TFLOPs"], "FP64 MFMA (FP32 weights, FP64 activations and accumulation)"
    elif args.precision == "fp8":
        peak, peak_name = PEAK["fp8_mfma_TFLOPs"], "FP8 MFMA (e4m3, FP32 accumulation)"
    else:
        peak, peak_name = PEAK["bf16_mfma_TFLOPs"], "BF16 MFMA"
    achieved = flops / recon_s / 1e12
    esz = {"fp32": 8, "bf16": 2, "fp8": 1}[args.precision]
    bytes_alg = model_bytes_per_leaf(model_bytes, H, W, esz, 24.0 if args.input5 else 8.0) * L
    ridge = peak * 1e12 / (PEAK["hbm_GBps"] * 1e9)
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{workload}_{args.precision}.json")
    src_sha = sha_of(os.path.join(ROOT, "paper_2010_01775_amd", "csrc", "net.hip"))
    if os.path.exists(tfile) and not args.experts and not args.input5:
        t = json.load(open(tfile))
        if t.get("source_sha") == src_sha:
            traffic = t.get("bytes_per_launch")

    stage_roof = {}
    for s_ in stages:
        if s_ == "recon":
            continue
        by = stage_bytes(s_, n_photons, L, H, W, nq, sorted_photons=pos is not None and args.hierarchy == "octree")
        gbps = by / (avg[s_] / 1e3) / 1e9
        stage_roof[s_] = {"ms": avg[s_], "algorithmic_bytes": by, "GBps": gbps, "frac_hbm": gbps / PEAK["hbm_GBps"]}
    stage_roof["recon"] = {"ms": avg["recon"], "algorithmic_flops": flops, "TFLOPs": achieved,
                           "frac_mfma": achieved / peak, "algorithmic_bytes": bytes_alg,
                           "frac_hbm": bytes_alg / recon_s / 1e9 / PEAK["hbm_GBps"]}

    res = {
        "metric": "leaf densities reconstructed/sec + guided samples/sec; p50/p99 batch latency",
        "value": L * args.steps / (total_ms / 1e3),
        "unit": "leaves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f64", "bf16": "bf16", "fp8": "fp8-e4m3"}[args.precision],
        "data": "synthetic (seeded vMF-mixture photons, He-init weights)",
        "config": {"workload": desc, "leaves": L, "photons": n_photons, "H": H, "W": W, "queries": nq,
                   "autotuned": tune,
                   "precision": {"fp32": "fp32 weights, f64 activations and conv accumulation",
                                 "bf16": "bf16 conv, f32 accumulation",
                                 "fp8": "fp8 e4m3 conv (static per-layer activation scales, "
                                        "per-output-channel weight scales), f32 accumulation"}[args.precision]}
                  | ({"fp8_calibration": calib} if calib else {})
                  | ({"experts": "5 U-Nets by leaf photon count [0,100) [100,500) [500,1000) [1000,5000) "
                                 "[5000,inf)", "expert_leaves": expert_leaves} if experts else {})
                  | ({"input": "5 channels: maps and photon counts of iterations t and t-1 (t-1: first half of "
                               "each leaf's photons), valid-bin mask; masked first layer"} if args.input5 else {})
                  | ({"network": "paper-style U-Net 16/32/64, ELU, residual links, bottleneck dilations 2 and 4, "
                                 "1x1 softplus head"} if args.paper_net else {}),
        "samples_per_s": nq / (avg["sample"] / 1e3),
        "eval_per_s": nq / (avg["eval"] / 1e3),
        **({"fused_form": fused} if fused else {}),
        "one_sample_mis": mis,
        "sampling_grouped_by_leaf": grouped,
        **({"kdgrid_locate": locate} if locate else {}),
        "p50_ms": float(np.percentile(per_step, 50)),
        "p99_ms": float(np.percentile(per_step, 99)),
        "stage_ms": avg,
        "stage_roofline": stage_roof,
        # the dominant stage: the network (a matrix-core contraction in every
        # precision; its HBM side beside it)
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": f"reconstruct_density (implicit-GEMM conv stack), {peak_name}",
                     "frac_is": "algorithmic FLOPs (direct 3x3 convolutions) per second over the peak",
                     "flops_per_launch": flops, "avg_launch_ms": avg["recon"],
                     "issued_flops_per_launch": mat_flops, "issued_TFLOPs": mat_flops / recon_s / 1e12,
                     "issued_frac": mat_flops / recon_s / 1e12 / peak,
                     "issued_is": "matrix-core FLOPs of the layers as launched (phase-merged decoder taps in "
                                  "FP32 mode) per second over the peak: the matrix-core utilisation",
                     "vector_flops_per_launch": vec_flops,
                     "bytes_per_launch": bytes_alg, "hbm_GBps": bytes_alg / recon_s / 1e9,
                     "hbm_frac": bytes_alg / recon_s / 1e9 / PEAK["hbm_GBps"],
                     "intensity_flop_per_byte": flops / bytes_alg, "ridge_flop_per_byte": ridge,
                     "source_sha": src_sha},
    }
    res["sampling_chi2"] = sampling_chi2(npg, ctx, tabs, L, H, W)
    if args.precision != "fp32":
        res["precision_vs_fp32"] = pdf_errors_vs_fp32(npg, ctx, model, energy, args.precision,
                                                      (count, *prev) if prev is not None else None)
    del sd, pe, q_leaf, q_u, dirs, w, energy, count, dens, tabs, hier_out, pos, prev
    for m in (experts or [model]):
        m.free()
    ctx.close()
    torch.cuda.empty_cache()
    if with_baseline and not args.no_cpu_baseline:
        if workload == "uniform":
            res["cpu_baseline"] = cpu_baseline_uniform(input5=args.input5,
                                                       model5=model_bytes if args.input5 else None)
        elif args.hierarchy == "octree" and not args.experts and not args.input5:
            res["cpu_baseline"] = cpu_baseline_clustered(cp, model_bytes, L, nq)
    return res


def calibrate_counters(nbytes: int = 1 << 30, reps: int = 8):
    """Copies of known size, for scaling HBM byte counters (run under
    rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE): each dispatch reads and
    writes exactly 2^30 bytes of a buffer 4x larger than the last-level
    cache, so a counter's bytes per dispatch over 2^30 is its scale."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": nbytes, "dispatches": reps}))


def measure_peaks():
    """What the chip delivers to library code, beside the published peaks
    the rooflines divide by: a 4 GiB device copy (HBM), and square GEMMs
    through torch (rocBLAS / hipBLASLt) in FP64, BF16 and, where torch has
    it, FP8 e4m3 with FP32 output. Context for the roofline fractions; the
    fractions themselves stay against the published peaks."""
    import torch
    dev = "cuda:0"
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / reps

    out = {}
    n = 1 << 30
    x = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
    y = torch.empty_like(x)
    t = timed(lambda: y.copy_(x), 10)
    out["hbm_copy_GBps"] = 2 * 4 * n / t / 1e9
    del x, y
    for name, dt, m in (("fp64_gemm_TFLOPs", torch.float64, 8192), ("bf16_gemm_TFLOPs", torch.bfloat16, 16384)):
        a = torch.randn(m, m, device=dev).to(dt)
        b = torch.randn(m, m, device=dev).to(dt)
        t = timed(lambda: torch.matmul(a, b), 5)
        out[name] = 2 * m ** 3 / t / 1e12
        del a, b
    try:
        m = 16384
        a = torch.randn(m, m, device=dev).to(torch.float8_e4m3fn)
        b = torch.randn(m, m, device=dev).to(torch.float8_e4m3fn).t()
        one = torch.ones((), device=dev)
        t = timed(lambda: torch._scaled_mm(a, b, scale_a=one, scale_b=one, out_dtype=torch.float32), 5)
        out["fp8_gemm_TFLOPs"] = 2 * m ** 3 / t / 1e12
    except Exception as e:   # FP8 GEMM not offered by this torch build
        out["fp8_gemm_TFLOPs"] = None
        out["fp8_note"] = f"{type(e).__name__}: {e}"[:200]
    out["published"] = {k: PEAK[k] for k in ("hbm_GBps", "fp64_mfma_TFLOPs", "bf16_mfma_TFLOPs", "fp8_mfma_TFLOPs")}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered", choices=["uniform", "clustered", "serving"],
                    help="clustered (default): 5e7 photons, octree, 128x128 maps, 1e8 samples; uniform: 1024 "
                         "leaves x 4096 photons, 64x64 maps, 2^20 samples; serving: the request stream")
    ap.add_argument("--no-extra", action="store_true",
                    help="clustered workload: skip the uniform batch that the default run times after it")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--experts", action="store_true",
                    help="five U-Nets chosen by leaf photon count ([0,100), [100,500), [500,1000), "
                         "[1000,5000), [5000,inf)) instead of one")
    ap.add_argument("--hierarchy", default="octree", choices=["octree", "kdgrid"],
                    help="clustered workload: the count-threshold octree, or the paper's hierarchical grid "
                         "(100^3 voxels, valid voxels from bounce points, local KD trees split by photon count "
                         "> 500 sqrt(2) or normal variance > 0.5, depth <= 8)")
    ap.add_argument("--paper-net", action="store_true",
                    help="the paper-style U-Net (16/32/64 channels, ELU, residual links, dilated bottleneck) "
                         "on the five-channel input (implies --input5)")
    ap.add_argument("--input5", action="store_true",
                    help="the five-channel network input (maps and photon counts of iterations t and t-1, "
                         "valid-bin mask) with a masked first layer; FP32 or BF16")
    ap.add_argument("--calibrate-counters", action="store_true",
                    help="only run 8 device copies of 1 GiB (for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure a 4 GiB copy and FP64/BF16/FP8 library GEMMs (context for the rooflines)")
    args = ap.parse_args()
    if args.calibrate_counters:
        return calibrate_counters()
    if args.peaks:
        return measure_peaks()
    if args.paper_net:
        args.input5 = True
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(leaves are independent; sharding them over GPUs is a design, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving":
        return run_serving(args)
    if args.input5 and (args.experts or args.precision == "fp8"):
        print("--input5 runs one five-channel U-Net in FP32 or BF16", file=sys.stderr)
        sys.exit(2)
    res = run_path(args, args.workload)
    if args.workload == "clustered" and not args.no_extra and args.hierarchy == "octree" and not args.experts \
            and not args.input5:
        # the uniform batch, timed the same way, as an extra key
        u = run_path(args, "uniform", with_baseline=not args.no_cpu_baseline)
        res["uniform_batch"] = {k: u[k] for k in ("value", "unit", "ms_per_step", "samples_per_s", "eval_per_s",
                                                  "fused_form", "sampling_grouped_by_leaf",
                                                  "p50_ms", "p99_ms", "stage_ms", "stage_roofline", "roofline",
                                                  "config", "sampling_chi2", "precision_vs_fp32", "cpu_baseline")
                                if k in u}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
