"""ctypes wrapper of the plain CPU FP64 oracle (npg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares no
code with the GPU path; both consume the same seeded inputs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "npg_oracle.c")
# NPG_ORACLE_SANITIZE=1 selects a separate build with AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload the ASan runtime)
SANITIZE = os.environ.get("NPG_ORACLE_SANITIZE") == "1"
LIB = os.path.join(HERE, "libnpg_oracle_san.so" if SANITIZE else "libnpg_oracle.so")

OK, E_ARG, E_RANGE, E_CAPACITY = 0, -1, -2, -3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        san = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined"] if SANITIZE else []
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", *san, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
        sig = {
            "or_boundaries": (None, [I, P, P]),
            "or_bin_dirs": (I, [P, I64, I, I, P]),
            "or_splat": (I, [P, P, P, P, I64, I, I, P, P, I]),
            "or_normalize_input": (None, [P, I64, I, I, P]),
            "or_net_forward": (I, [P, C.c_size_t, P, I64, I, I, P]),
            "or_conv2d": (None, [P, P, I, I, I, P, I, I, P]),
            "or_conv2d_dil": (None, [P, P, I, I, I, P, I, I, I, P]),
            "or_net_forward5": (I, [P, C.c_size_t, P, I64, I, I, P]),
            "or_input5": (None, [P, P, P, P, I64, I, I, P]),
            "or_pconv2d": (None, [P, P, I, I, I, P, I, I, I, P]),
            "or_build_cdf": (I, [P, I64, I, I, P, P, P, P]),
            "or_sample": (I, [P, P, P, I64, I, I, P, P, I64, P, P, P]),
            "or_eval_pdf": (I, [P, I64, I, I, P, P, I64, P]),
            "or_build_tree": (I, [P, I64, C.c_uint32, I, P, P, P, P, P, I64, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def boundaries(W: int):
    ex = np.empty(W, np.float32)
    ey = np.empty(W, np.float32)
    lib().or_boundaries(W, _p(ex), _p(ey))
    return ex, ey


def bin_dirs(dirs, H: int, W: int):
    dirs = _c(dirs, np.float32)
    out = np.empty(dirs.shape[0], np.int32)
    rc = lib().or_bin_dirs(_p(dirs), dirs.shape[0], H, W, _p(out))
    return rc, out


def splat(dirs, w, leaf_off, H, W, perm=None, energy=None, count=None, accumulate=False,
          want_count=True):
    dirs = _c(dirs, np.float32)
    w = _c(w, np.uint32)
    leaf_off = _c(leaf_off, np.uint32)
    L = leaf_off.shape[0] - 1
    if energy is None:
        energy = np.zeros((L, H, W), np.uint64)
    if count is None and want_count:
        count = np.zeros((L, H, W), np.uint32)
    perm = None if perm is None else _c(perm, np.uint32)
    rc = lib().or_splat(_p(dirs), _p(w), _p(perm), _p(leaf_off), L, H, W, _p(energy),
                        _p(count), int(bool(accumulate)))
    return rc, energy, count


def normalize_input(energy):
    energy = _c(energy, np.uint64)
    L, H, W = energy.shape
    x = np.empty((L, H, W), np.float64)
    lib().or_normalize_input(_p(energy), L, H, W, _p(x))
    return x


def net_forward(model: bytes, x):
    x = _c(x, np.float64)
    L, H, W = x.shape
    s = np.empty((L, H, W), np.float64)
    buf = np.frombuffer(model, dtype=np.uint8)
    rc = lib().or_net_forward(_p(buf), len(model), _p(x), L, H, W, _p(s))
    return rc, s


def expert_of(photons, bounds):
    """Mixture of experts by photon count (Sec. 8, Implementation, training):
    expert e is responsible for the range [lo_e, hi_e) of photons per voxel,
    lo_0 = 0, lo_e = bounds[e-1], hi_e = bounds[e], hi_last = infinity.
    Returns, per count, the index of the range that holds it."""
    los = [0] + [int(b) for b in bounds]
    his = [int(b) for b in bounds] + [None]
    out = []
    for n in np.asarray(photons).ravel().tolist():
        e = next(i for i, (lo, hi) in enumerate(zip(los, his)) if lo <= n and (hi is None or n < hi))
        out.append(e)
    return np.array(out, dtype=np.int64)


def experts_forward(models, photons, bounds, x):
    """Each leaf's map through the network of its expert (net_forward per
    expert on that expert's leaves)."""
    x = _c(x, np.float64)
    e = expert_of(photons, bounds)
    out = np.empty_like(x)
    for k, model in enumerate(models):
        sel = np.nonzero(e == k)[0]
        if sel.size:
            rc, out[sel] = net_forward(model, x[sel])
            if rc:
                return rc, out
    return OK, out


def conv2d(w, b, x):
    """One conv layer: w [co,ci,k,k] f32, b [co] f32 or None, x [ci,H,W] f64."""
    w = _c(w, np.float32)
    co, ci, k, _ = w.shape
    x = _c(x, np.float64)
    _, H, W = x.shape
    out = np.empty((co, H, W), np.float64)
    bb = None if b is None else _c(b, np.float32)
    lib().or_conv2d(_p(w), _p(bb), co, ci, k, _p(x), H, W, _p(out))
    return out


def conv2d_dil(w, b, x, dil):
    """One conv layer with dilation `dil` (taps at offsets of dil pixels)."""
    w = _c(w, np.float32)
    co, ci, k, _ = w.shape
    x = _c(x, np.float64)
    _, H, W = x.shape
    out = np.empty((co, H, W), np.float64)
    bb = None if b is None else _c(b, np.float32)
    lib().or_conv2d_dil(_p(w), _p(bb), co, ci, k, _p(x), int(dil), H, W, _p(out))
    return out


def pconv2d(w, b, x, mask_ch):
    """One masked (partial) conv layer with the mask in channel mask_ch of
    x [ci,H,W] (the paper's first layer, Sec. 6.1)."""
    w = _c(w, np.float32)
    co, ci, k, _ = w.shape
    x = _c(x, np.float64)
    _, H, W = x.shape
    out = np.empty((co, H, W), np.float64)
    bb = None if b is None else _c(b, np.float32)
    lib().or_pconv2d(_p(w), _p(bb), co, ci, k, _p(x), int(mask_ch), H, W, _p(out))
    return out


def input5(e_t, e_p, p_t, p_p):
    """The five input channels (Sec. 6): raw maps of iterations t and t-1,
    their photon counts (each mean-1 normalised, float32-rounded) and the
    mask of bins with photons at t.  Returns x [L][5][H][W] (float64)."""
    e_t, e_p = _c(e_t, np.uint64), _c(e_p, np.uint64)
    p_t, p_p = _c(p_t, np.uint32), _c(p_p, np.uint32)
    L, H, W = e_t.shape
    x = np.empty((L, 5, H, W), np.float64)
    lib().or_input5(_p(e_t), _p(e_p), _p(p_t), _p(p_p), L, H, W, _p(x))
    return x


def net_forward5(model: bytes, x):
    """Five-channel U-Net (masked first layer) on x [L][5][H][W]."""
    x = _c(x, np.float64)
    L, _, H, W = x.shape
    s = np.empty((L, H, W), np.float64)
    buf = np.frombuffer(model, dtype=np.uint8)
    rc = lib().or_net_forward5(_p(buf), len(model), _p(x), L, H, W, _p(s))
    return rc, s


def build_cdf(s):
    s = _c(s, np.float64)
    L, H, W = s.shape
    pdf = np.empty((L, H, W), np.float32)
    marg = np.empty((L, H + 1), np.float32)
    cond = np.empty((L, H, W + 1), np.float32)
    total = np.empty(L, np.float64)
    rc = lib().or_build_cdf(_p(s), L, H, W, _p(pdf), _p(marg), _p(cond), _p(total))
    return rc, pdf, marg, cond, total


def sample(pdf, marg, cond, leaf, u):
    pdf = _c(pdf, np.float32)
    marg = _c(marg, np.float32)
    cond = _c(cond, np.float32)
    L, H, W = pdf.shape
    leaf = _c(leaf, np.uint32)
    u = _c(u, np.float32)
    n = leaf.shape[0]
    d = np.empty((n, 3), np.float64)
    p = np.empty(n, np.float32)
    b = np.empty(n, np.uint32)
    rc = lib().or_sample(_p(pdf), _p(marg), _p(cond), L, H, W, _p(leaf), _p(u), n, _p(d), _p(p), _p(b))
    return rc, d, p, b


def eval_pdf(pdf, leaf, dirs):
    pdf = _c(pdf, np.float32)
    L, H, W = pdf.shape
    leaf = _c(leaf, np.uint32)
    dirs = _c(dirs, np.float32)
    n = leaf.shape[0]
    out = np.empty(n, np.float32)
    rc = lib().or_eval_pdf(_p(pdf), L, H, W, _p(leaf), _p(dirs), n, _p(out))
    return rc, out


# ------------------------------------------------------- one-sample MIS
MIS_MIN_PATHS = 50          # both strategies need this many bounces (Sec. 7.3)
MIS_CLAMP = (0.2, 0.8)      # alpha is clamped to this range (Sec. 7.3)


def mis_alpha(nu_b, nu_g, q_b, q_g):
    """Eq. mis_alpha: alpha_j = nu_bar_B / (nu_bar_B + nu_bar_G), nu_bar =
    nu / Q, once Q_B and Q_G reach MIS_MIN_PATHS (0.5 before, and 0.5 when
    both averages are zero), clamped to MIS_CLAMP; binary64, stored as
    float32.  Returns (rc, alpha); a negative or non-finite contribution
    gives E_RANGE and 0.5 for that leaf."""
    out = []
    rc = OK
    for nb, ng, qb, qg in zip(np.asarray(nu_b, np.float64).tolist(), np.asarray(nu_g, np.float64).tolist(),
                              np.asarray(q_b).tolist(), np.asarray(q_g).tolist()):
        if not (np.isfinite(nb) and np.isfinite(ng) and nb >= 0.0 and ng >= 0.0):
            rc = E_RANGE
            out.append(0.5)
            continue
        a = 0.5
        if qb >= MIS_MIN_PATHS and qg >= MIS_MIN_PATHS:
            mb, mg = nb / qb, ng / qg
            if mb + mg > 0.0:
                a = mb / (mb + mg)
        out.append(min(max(a, MIS_CLAMP[0]), MIS_CLAMP[1]))
    return rc, np.array(out, dtype=np.float32)


def onb(n):
    """Orthonormal frame (t, b) completing the unit normal n (Duff et al.,
    Building an Orthonormal Basis, Revisited, JCGT 6(1), 2017)."""
    n = np.asarray(n, np.float64)
    nx, ny, nz = n[:, 0], n[:, 1], n[:, 2]
    sign = np.where(nz >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + nz)
    b = nx * ny * a
    t = np.stack([1.0 + sign * nx * nx * a, sign * b, -sign * nx], axis=1)
    bt = np.stack([b, sign + ny * ny * a, -ny], axis=1)
    return t, bt


def cosine_sample(n, u1, u2):
    """Cosine-weighted direction about n: disk point (sqrt(u1), 2 pi u2)
    lifted to the hemisphere (Malley's method)."""
    n = np.asarray(n, np.float64)
    u1 = np.asarray(u1, np.float64)
    u2 = np.asarray(u2, np.float64)
    t, bt = onb(n)
    r = np.sqrt(u1)
    phi = 2.0 * np.pi * u2
    h = np.sqrt(np.maximum(0.0, 1.0 - u1))
    return (r * np.cos(phi))[:, None] * t + (r * np.sin(phi))[:, None] * bt + h[:, None] * n


def cosine_pdf(n, w):
    """p_BSDF of the cosine lobe: max(0, n.w) / pi."""
    c = np.sum(np.asarray(n, np.float64) * np.asarray(w, np.float64), axis=1)
    return np.maximum(0.0, c) / np.pi


def eval_pdf_mis(pdf, alpha, leaf, normal, dirs):
    """Eq. mis_coef: a p_BSDF(w) + (1 - a) pdf[l][bin(w)], a = alpha[l]."""
    a = np.asarray(alpha, np.float64)[np.asarray(leaf, np.int64)]
    rc, g = eval_pdf(pdf, leaf, dirs)
    return rc, a * cosine_pdf(normal, dirs) + (1.0 - a) * g.astype(np.float64)


def sample_mis(pdf, marg, cond, alpha, leaf, normal, u):
    """One-sample MIS: u0 < alpha[l] picks the BSDF (cosine lobe from
    (u1, u2)), else the guided sample of `sample` from (u1, u2); the pdf is
    the mixture, with the guide term of the sampled bin for guided samples
    and of bin(w) (w rounded to float32) for BSDF samples.  Returns
    (rc, dirs, pdf, strategy) with strategy 1 = BSDF."""
    u = np.asarray(u, np.float32)
    leaf = np.asarray(leaf, np.uint32)
    alpha = np.asarray(alpha, np.float32)
    n = u.shape[0]
    L = pdf.shape[0]
    ok = leaf < L
    a32 = np.where(ok, alpha[np.minimum(leaf, L - 1)], np.float32(0))
    strat = (u[:, 0] < a32).astype(np.uint8)
    rc, dg, pg, bg = sample(pdf, marg, cond, leaf, u[:, 1:3])
    db = cosine_sample(normal, u[:, 1], u[:, 2])
    d = np.where(strat[:, None] == 1, db, dg)
    a = a32.astype(np.float64)
    pb = cosine_pdf(normal, d)
    rc2, g_b = eval_pdf(pdf, np.minimum(leaf, L - 1), d.astype(np.float32))
    g = np.where(strat == 1, g_b.astype(np.float64), pg.astype(np.float64))
    p = a * pb + (1.0 - a) * g
    bad = ~ok | ~np.all((u >= 0) & (u < 1), axis=1) | ~np.all(np.isfinite(normal), axis=1)
    d[bad] = np.nan
    p[bad] = np.nan
    if np.any(bad):
        rc = E_RANGE
    return rc, d, p, strat


def build_tree(pos, T: int = 8192, Dmax: int = 6, max_leaves: int | None = None):
    pos = _c(pos, np.float32)
    n = pos.shape[0]
    if max_leaves is None:
        max_leaves = max(1, n)
    perm = np.empty(max(n, 1), np.uint32)
    leaf_of = np.empty(max(n, 1), np.uint32)
    off = np.zeros(max_leaves + 1, np.uint32)
    key = np.zeros(max_leaves, np.uint64)
    depth = np.zeros(max_leaves, np.uint8)
    nl = C.c_int64(0)
    rc = lib().or_build_tree(_p(pos), n, T, Dmax, _p(perm), _p(leaf_of), _p(off), _p(key),
                             _p(depth), max_leaves, C.addressof(nl))
    L = min(nl.value, max_leaves)
    return rc, dict(perm=perm[:n], leaf_of=leaf_of[:n], leaf_off=off[:L + 1], key=key[:L],
                    depth=depth[:L], n_leaves=nl.value)


def pipeline(batch, want_tables=True):
    """The full oracle chain on a leaf batch: splat -> normalise -> net -> CDF."""
    rc, E, P = splat(batch.dirs, batch.w, batch.leaf_off, batch.H, batch.W)
    assert rc == OK
    x = normalize_input(E)
    rc, s = net_forward(batch.model, x)
    assert rc == OK
    rc, pdf, marg, cond, total = build_cdf(s)
    return dict(energy=E, count=P, x=x, s=s, pdf=pdf, marg=marg, cond=cond, total=total)
