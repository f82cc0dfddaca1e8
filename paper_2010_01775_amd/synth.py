"""Seeded synthetic inputs for the photon-guiding hot path.

This module holds none of the method's arithmetic.  It only draws the random
inputs that the GPU library and the CPU oracle both consume:

* photon directions from von Mises-Fisher (vMF) mixtures on the unit sphere,
* photon weights (lognormal flux, quantised to uint32 in units of 2^-16),
* clustered photon positions in the unit box,
* guided-sampling queries (leaf id + two uniforms),
* He-normal network weights, serialised in the ``NPGW`` weight-file format.

The paper's scenes, datasets and trained weights are not available; these
draws stand in for them with the shapes the paper reports (a few to a few
thousand photons per voxel, thousands of voxels, 2D maps of a few thousand
bins) scaled up to the sizes of the benchmark workloads.

Random numbers: numpy PCG64 seeded per workload.  vMF sampling follows the
numerically stable inverse CDF of Wood (1994) as written by Jakob (2012,
"Numerically stable sampling of the von Mises Fisher distribution on S^2");
tangent frames use Duff et al. (2017, "Building an orthonormal basis,
revisited").
"""
from __future__ import annotations

import struct
from dataclasses import dataclass, field

import numpy as np

U24 = np.float32(2.0 ** -24)
W_UNIT = 65536.0  # photon weights are stored in units of 2^-16
U32_MAX = 2 ** 32 - 1


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniforms(rng: np.random.Generator, n: int) -> np.ndarray:
    """n float32 uniforms in [0, 1): (u32 >> 8) * 2^-24, exact in float32."""
    r = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64) >> np.uint64(8)
    return r.astype(np.float32) * U24


def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    """n directions uniform on S^2 (normalised Gaussians), float64 [n,3]."""
    v = rng.standard_normal((n, 3))
    nrm = np.linalg.norm(v, axis=1, keepdims=True)
    bad = nrm[:, 0] < 1e-12
    while bad.any():
        v[bad] = rng.standard_normal((int(bad.sum()), 3))
        nrm = np.linalg.norm(v, axis=1, keepdims=True)
        bad = nrm[:, 0] < 1e-12
    return v / nrm


def _onb(mu: np.ndarray):
    """Orthonormal tangents (t1, t2) for unit vectors mu [n,3] (Duff et al.)."""
    x, y, z = mu[:, 0], mu[:, 1], mu[:, 2]
    sgn = np.where(z >= 0.0, 1.0, -1.0)
    a = -1.0 / (sgn + z)
    b = x * y * a
    t1 = np.stack([1.0 + sgn * x * x * a, sgn * b, -sgn * x], axis=1)
    t2 = np.stack([b, sgn + y * y * a, -y], axis=1)
    return t1, t2


def vmf_directions(rng: np.random.Generator, mu: np.ndarray, kappa: np.ndarray) -> np.ndarray:
    """One vMF draw per row: mean mu [n,3] (unit), concentration kappa [n] > 0.

    Returns float64 [n,3].  Cosine to the mean: w = 1 + ln(u + (1-u) e^{-2k}) / k.
    """
    n = mu.shape[0]
    u = rng.random(n)
    psi = 2.0 * np.pi * rng.random(n)
    w = 1.0 + np.log(u + (1.0 - u) * np.exp(-2.0 * kappa)) / kappa
    w = np.clip(w, -1.0, 1.0)
    r = np.sqrt(np.maximum(0.0, 1.0 - w * w))
    t1, t2 = _onb(mu)
    return (r * np.cos(psi))[:, None] * t1 + (r * np.sin(psi))[:, None] * t2 + w[:, None] * mu


def to_f32_dirs(d: np.ndarray) -> np.ndarray:
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    return np.ascontiguousarray(d.astype(np.float32))


def photon_weights(rng: np.random.Generator, n: int) -> np.ndarray:
    """Lognormal(0, 0.5) flux, quantised: w = min(2^32-1, rint(x * 2^16))."""
    x = rng.lognormal(0.0, 0.5, n)
    return np.minimum(np.rint(x * W_UNIT), U32_MAX).astype(np.uint32)


def two_lobe_mixture(rng: np.random.Generator, n: int, mu1, mu2,
                     k1: float = 20.0, k2: float = 200.0,
                     p=(0.6, 0.3, 0.1)) -> np.ndarray:
    """n directions from p0 vMF(k1, mu1) + p1 vMF(k2, mu2) + p2 uniform (float32)."""
    comp = rng.choice(3, size=n, p=np.asarray(p, dtype=np.float64))
    mu = np.empty((n, 3))
    kap = np.ones(n)
    mu[comp == 0] = mu1
    kap[comp == 0] = k1
    mu[comp == 1] = mu2
    kap[comp == 1] = k2
    out = np.empty((n, 3))
    lobe = comp < 2
    out[lobe] = vmf_directions(rng, mu[lobe], kap[lobe])
    out[~lobe] = unit_vectors(rng, int((~lobe).sum()))
    return to_f32_dirs(out)


# --------------------------------------------------------------------------
# Network weights (NPGW file)
# --------------------------------------------------------------------------
ARCH_CNN = 1
ARCH_UNET = 2
ARCH_PAPER = 3


def cnn_layers(channels=(1, 16, 16, 1)):
    """(cout, cin, k) of a plain 3x3 conv chain."""
    return [(channels[i + 1], channels[i], 3) for i in range(len(channels) - 1)]


def unet_layers(levels=(16, 32, 64, 128), cin: int = 1):
    """(cout, cin, k) of the U-Net in file order.

    Encoder level d: two 3x3 convs (in -> c_d -> c_d).  Decoder level d
    (from the second-deepest up): two 3x3 convs on [upsampled, skip] channels
    (c_{d+1} + c_d -> c_d -> c_d).  Head: 1x1 conv c_0 -> 1.
    """
    out = []
    prev = cin
    for c in levels:
        out += [(c, prev, 3), (c, c, 3)]
        prev = c
    for d in range(len(levels) - 2, -1, -1):
        c = levels[d]
        out += [(c, levels[d + 1] + c, 3), (c, c, 3)]
    out.append((1, levels[0], 1))
    return out


def paper_unet_layers(levels=(16, 32, 64), cin: int = 5):
    """(cout, cin, k) of the paper-style U-Net in file order.

    Encoder level d (not the deepest): two 3x3 convs (in -> c_d -> c_d).
    Deepest level: one 3x3 conv and two dilated 3x3 convs (c -> c -> c).
    Decoder level d: two 3x3 convs (c_{d+1} + c_d -> c_d -> c_d).  Head:
    1x1 conv c_0 -> 1.
    """
    out = []
    prev = cin
    for i, c in enumerate(levels):
        out += [(c, prev, 3)] + [(c, c, 3)] * (2 if i == len(levels) - 1 else 1)
        prev = c
    for d in range(len(levels) - 2, -1, -1):
        c = levels[d]
        out += [(c, levels[d + 1] + c, 3), (c, c, 3)]
    out.append((1, levels[0], 1))
    return out


def he_weights(seed: int, layers, random_bias: bool = False):
    """He-normal N(0, 2/fan_in) weights, OIHW, drawn in layer order; zero biases."""
    rng = rng_for(seed)
    ws, bs = [], []
    for (co, ci, k) in layers:
        std = np.sqrt(2.0 / (ci * k * k))
        w = (rng.standard_normal((co, ci, k, k)) * std).astype(np.float32)
        if random_bias:
            b = (rng.standard_normal(co) * 0.1).astype(np.float32)
        else:
            b = np.zeros(co, dtype=np.float32)
        ws.append(w)
        bs.append(b)
    return ws, bs


def pack_model(arch: int, levels: int, ws, bs) -> bytes:
    """Serialise to the NPGW v1 little-endian format.

    magic 'NPGW' | u32 version=1 | u32 arch | u32 levels | u32 n_layers |
    per layer: u32 cout, u32 cin, u32 k, f32 w[cout][cin][k][k], f32 b[cout]
    """
    parts = [b"NPGW", struct.pack("<IIII", 1, arch, levels, len(ws))]
    for w, b in zip(ws, bs):
        co, ci, k, k2 = w.shape
        assert k == k2 and b.shape == (co,)
        parts.append(struct.pack("<III", co, ci, k))
        parts.append(np.ascontiguousarray(w, dtype="<f4").tobytes())
        parts.append(np.ascontiguousarray(b, dtype="<f4").tobytes())
    return b"".join(parts)


def cnn_model(seed: int, channels=(1, 16, 16, 1), random_bias=False) -> bytes:
    ws, bs = he_weights(seed, cnn_layers(channels), random_bias)
    return pack_model(ARCH_CNN, 0, ws, bs)


def unet_model(seed: int, levels=(16, 32, 64, 128), random_bias=False) -> bytes:
    ws, bs = he_weights(seed, unet_layers(levels), random_bias)
    return pack_model(ARCH_UNET, len(levels), ws, bs)


def unet5_model(seed: int, levels=(16, 32, 64, 128), random_bias=False) -> bytes:
    """The U-Net with the five input channels of the paper (masked first layer)."""
    ws, bs = he_weights(seed, unet_layers(levels, cin=5), random_bias)
    return pack_model(ARCH_UNET, len(levels), ws, bs)


def paper_unet_model(seed: int, levels=(16, 32, 64), random_bias=False) -> bytes:
    """The paper-style U-Net (five input channels, ELU, residual links,
    dilated bottleneck), He-init stand-in weights."""
    ws, bs = he_weights(seed, paper_unet_layers(levels), random_bias)
    return pack_model(ARCH_PAPER, len(levels), ws, bs)


def surface_normals(seed: int, pos: np.ndarray, n_creases: int = 16, crease_radius: float = 0.1,
                    freq: float = 1.5, jitter: float = 0.05, chunk: int = 5_000_000) -> np.ndarray:
    """Unit surface normals at photon hit points, float32 [n,3].

    A smooth random field, normalize(c + sum_k a_k sin(2 pi freq (w_k . p) + phi_k))
    with four random plane waves, so that normals vary slowly over the
    scene; plus n_creases crease discs (random centre, plane and radius
    crease_radius) across which the normal flips sign, standing in for the
    geometric edges where normals change abruptly; plus Gaussian jitter
    (std `jitter` per component), renormalised.
    """
    rng = rng_for(seed)
    c = unit_vectors(rng, 1)[0]
    a = 0.6 * rng.standard_normal((4, 3))
    wv = unit_vectors(rng, 4)
    ph = rng.uniform(0.0, 2.0 * np.pi, 4)
    cc = rng.random((n_creases, 3))
    cm = unit_vectors(rng, n_creases)
    out = np.empty((pos.shape[0], 3), np.float32)
    for s0 in range(0, pos.shape[0], chunk):
        p = pos[s0:s0 + chunk].astype(np.float64)
        v = np.tile(c, (p.shape[0], 1))
        for k in range(4):
            v += a[k] * np.sin(2.0 * np.pi * freq * (p @ wv[k]) + ph[k])[:, None]
        nv = np.linalg.norm(v, axis=1, keepdims=True)
        v = np.where(nv > 1e-6, v / np.maximum(nv, 1e-300), c)
        for j in range(n_creases):
            d = p - cc[j]
            far = (np.einsum("ij,ij->i", d, d) < crease_radius ** 2) & (d @ cm[j] > 0)
            v[far] = -v[far]
        v = v + jitter * rng.standard_normal((p.shape[0], 3))
        out[s0:s0 + chunk] = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    return out


def bounce_points(seed: int, pos: np.ndarray, n: int, spread: float = 0.01) -> np.ndarray:
    """Stand-ins for the bounce points of camera paths, float32 [n,3]: random
    photon positions moved by Gaussian noise of std `spread`, clipped to the
    unit box (camera paths reach roughly where photons land)."""
    rng = rng_for(seed)
    i = rng.integers(0, pos.shape[0], n)
    p = pos[i].astype(np.float64) + spread * rng.standard_normal((n, 3))
    return np.clip(p, 0.0, np.nextafter(1.0, 0.0)).astype(np.float32)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
@dataclass
class LeafBatch:
    """Photons already grouped by leaf (CSR), plus queries."""
    H: int
    W: int
    dirs: np.ndarray          # f32 [N,3]
    w: np.ndarray             # u32 [N]
    leaf_off: np.ndarray      # u32 [L+1]
    q_leaf: np.ndarray        # u32 [Q]
    q_u: np.ndarray           # f32 [Q,2]
    model: bytes
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def L(self) -> int:
        return int(self.leaf_off.shape[0] - 1)


def single_leaf(seed: int = 1000, n: int = 4096, H: int = 32, W: int = 32,
                n_queries: int = 65536) -> LeafBatch:
    """One leaf: 0.6 vMF(20) + 0.3 vMF(200) + 0.1 uniform, 3-layer CNN."""
    rng = rng_for(seed)
    mus = unit_vectors(rng, 2)
    dirs = two_lobe_mixture(rng, n, mus[0], mus[1])
    w = photon_weights(rng, n)
    q_u = np.stack([uniforms(rng, n_queries), uniforms(rng, n_queries)], axis=1)
    return LeafBatch(H, W, dirs, w, np.array([0, n], dtype=np.uint32),
                     np.zeros(n_queries, dtype=np.uint32), np.ascontiguousarray(q_u),
                     cnn_model(seed), seed, {"mu": mus})


def uniform_batch(seed: int = 1001, L: int = 1024, per_leaf: int = 4096,
                  H: int = 64, W: int = 64, n_queries: int = 1 << 20,
                  model: bytes | None = None) -> LeafBatch:
    """L leaves x per_leaf photons, each leaf with its own two lobes; U-Net."""
    rng = rng_for(seed)
    mus = unit_vectors(rng, 2 * L).reshape(L, 2, 3)
    n = L * per_leaf
    comp = rng.choice(3, size=n, p=[0.6, 0.3, 0.1])
    leaf = np.repeat(np.arange(L), per_leaf)
    mu = np.where((comp == 0)[:, None], mus[leaf, 0], mus[leaf, 1])
    kap = np.where(comp == 0, 20.0, 200.0)
    d = vmf_directions(rng, mu, kap)
    uni = comp == 2
    d[uni] = unit_vectors(rng, int(uni.sum()))
    dirs = to_f32_dirs(d)
    w = photon_weights(rng, n)
    off = (np.arange(L + 1, dtype=np.uint64) * per_leaf).astype(np.uint32)
    q_leaf = rng.integers(0, L, size=n_queries, dtype=np.uint32)
    q_u = np.stack([uniforms(rng, n_queries), uniforms(rng, n_queries)], axis=1)
    if model is None:
        model = unet_model(seed)
    return LeafBatch(H, W, dirs, w, off, q_leaf, np.ascontiguousarray(q_u), model, seed)


@dataclass
class ClusteredPhotons:
    """Photons in original (trace) order: positions, directions, weights."""
    pos: np.ndarray    # f32 [N,3] in [0,1)^3
    dirs: np.ndarray   # f32 [N,3]
    w: np.ndarray      # u32 [N]
    seed: int
    meta: dict = field(default_factory=dict)


def clustered_photons(seed: int = 1002, n: int = 50_000_000, n_clusters: int = 64,
                      sigma=(0.01, 0.1), cell_res: int = 64,
                      chunk: int = 5_000_000) -> ClusteredPhotons:
    """Photons from isotropic Gaussian clusters in the unit box.

    Cluster centres U[0,1)^3, sigma log-uniform, equal photon share; draws
    outside [0,1)^3 (after rounding to float32) are redrawn; the final order
    is a random permutation (photons arrive in trace order, not by cluster).
    Directions: each cell of a fixed cell_res^3 grid owns a vMF mixture with
    U{1..4} lobes, kappa log-uniform [5,500], Dirichlet(1) lobe weights; a
    photon draws from the mixture of the cell containing it.
    """
    rng = rng_for(seed)
    centres = rng.random((n_clusters, 3))
    sig = np.exp(rng.uniform(np.log(sigma[0]), np.log(sigma[1]), n_clusters))
    share = np.full(n_clusters, n // n_clusters, dtype=np.int64)
    share[: n - int(share.sum())] += 1
    pos = np.empty((n, 3), dtype=np.float32)
    o = 0
    for c in range(n_clusters):
        m = int(share[c])
        fill = 0
        while fill < m:
            need = m - fill
            p = (centres[c] + sig[c] * rng.standard_normal((need + need // 8 + 16, 3))).astype(np.float32)
            ok = np.all((p >= 0.0) & (p < 1.0), axis=1)
            p = p[ok][:need]
            pos[o + fill:o + fill + p.shape[0]] = p
            fill += p.shape[0]
        o += m
    order = rng.permutation(n)
    pos = pos[order]

    ncell = cell_res ** 3
    n_lobes = rng.integers(1, 5, size=ncell)
    lobe_mu = unit_vectors(rng, ncell * 4).reshape(ncell, 4, 3)
    lobe_k = np.exp(rng.uniform(np.log(5.0), np.log(500.0), (ncell, 4)))
    g = rng.standard_gamma(1.0, (ncell, 4))
    g[np.arange(4)[None, :] >= n_lobes[:, None]] = 0.0
    lobe_p = g / g.sum(axis=1, keepdims=True)
    lobe_cdf = np.cumsum(lobe_p, axis=1)
    lobe_cdf[np.arange(ncell), n_lobes - 1] = 1.0

    dirs = np.empty((n, 3), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        ci = np.minimum((pos[s:e].astype(np.float64) * cell_res).astype(np.int64), cell_res - 1)
        cell = ci[:, 0] + cell_res * (ci[:, 1] + cell_res * ci[:, 2])
        u = rng.random(e - s)
        lobe = (u[:, None] >= lobe_cdf[cell]).sum(axis=1)
        lobe = np.minimum(lobe, n_lobes[cell] - 1)
        d = vmf_directions(rng, lobe_mu[cell, lobe], lobe_k[cell, lobe])
        dirs[s:e] = to_f32_dirs(d)
    w = photon_weights(rng, n)
    return ClusteredPhotons(pos, dirs, w, seed,
                            {"centres": centres, "sigma": sig, "cell_res": cell_res})


def queries(seed: int, L: int, n: int):
    """n guided-sampling queries: leaf uniform over [0, L), two float32 uniforms."""
    rng = rng_for(seed)
    q_leaf = rng.integers(0, L, size=n, dtype=np.uint32)
    q_u = np.stack([uniforms(rng, n), uniforms(rng, n)], axis=1)
    return q_leaf, np.ascontiguousarray(q_u)


def random_density(seed: int, L: int, H: int, W: int, zero_frac: float = 0.0) -> np.ndarray:
    """A positive float32 density [L,H,W] (lognormal), optionally with zero bins/rows."""
    rng = rng_for(seed)
    s = rng.lognormal(0.0, 1.5, (L, H, W)).astype(np.float32)
    if zero_frac > 0.0:
        s[rng.random((L, H, W)) < zero_frac] = 0.0
    return s


# --------------------------------------------------------------------------
# Serving stream
# --------------------------------------------------------------------------
@dataclass
class Request:
    kind: str            # "recon" or "sample"
    t_arrive: float      # seconds from stream start
    H: int = 0
    W: int = 0
    n_leaves: int = 0
    counts: np.ndarray | None = None   # photons per leaf
    n_queries: int = 0
    seed: int = 0


def serving_stream(seed: int = 1004, n_requests: int = 2000, rate_hz: float = 100.0,
                   max_leaves: int = 4096, photons=(9.68, 1.38, 256, 1_000_000),
                   qrange=(1e4, 1e7)):
    """Poisson arrivals; reconstruction and sampling requests interleaved 1:1."""
    rng = rng_for(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n_requests))
    out = []
    for i in range(n_requests):
        if i % 2 == 0:
            nl = int(np.floor(np.exp(rng.uniform(0.0, np.log(max_leaves + 1)))))
            nl = max(1, min(max_leaves, nl))
            c = np.exp(rng.normal(photons[0], photons[1], nl))
            bad = (c < photons[2]) | (c > photons[3])
            while bad.any():
                c[bad] = np.exp(rng.normal(photons[0], photons[1], int(bad.sum())))
                bad = (c < photons[2]) | (c > photons[3])
            grid = 64 if rng.random() < 0.5 else 128
            out.append(Request("recon", float(t[i]), grid, grid, nl,
                               c.astype(np.int64), 0, int(rng.integers(0, 2 ** 31))))
        else:
            nq = int(np.exp(rng.uniform(np.log(qrange[0]), np.log(qrange[1]))))
            out.append(Request("sample", float(t[i]), n_queries=nq,
                               seed=int(rng.integers(0, 2 ** 31))))
    return out


def request_photons(req: Request):
    """Directions and weights for a reconstruction request (leaf-sorted, CSR)."""
    rng = rng_for(req.seed)
    L = req.n_leaves
    counts = req.counts
    off = np.zeros(L + 1, dtype=np.uint64)
    off[1:] = np.cumsum(counts)
    n = int(off[-1])
    mus = unit_vectors(rng, 2 * L).reshape(L, 2, 3)
    leaf = np.repeat(np.arange(L), counts)
    comp = rng.choice(3, size=n, p=[0.6, 0.3, 0.1])
    mu = np.where((comp == 0)[:, None], mus[leaf, 0], mus[leaf, 1])
    kap = np.where(comp == 0, 20.0, 200.0)
    d = vmf_directions(rng, mu, kap)
    uni = comp == 2
    d[uni] = unit_vectors(rng, int(uni.sum()))
    return to_f32_dirs(d), photon_weights(rng, n), off.astype(np.uint32)
