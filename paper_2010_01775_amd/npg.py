"""Python binding of libnpg.so (the C-ABI in include/npg.h).

Argument marshalling only: every step runs in the library's HIP kernels.
torch tensors provide device memory and the current stream.  Importing this
module does not need a GPU; loading the library does, and fails loudly if the
library has not been built (``python -m paper_2010_01775_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnpg.so")

OK, E_ARG, E_RANGE, E_CAPACITY, E_BUDGET, E_HIP = 0, -1, -2, -3, -4, -5
FP32, BF16, FP8 = 0, 1, 2
PRECISION = {"fp32": FP32, "bf16": BF16, "fp8": FP8}

SYMBOLS = [
    "npg_create", "npg_destroy", "npg_last_error", "npg_sync_status", "npg_memory_usage", "npg_conv_flops",
    "npg_model_load", "npg_model_free", "npg_model_calibrate_fp8",
    "npg_build_hierarchy", "npg_build_hierarchy_sorted", "npg_mark_valid", "npg_build_kdgrid", "npg_locate",
    "npg_splat_histograms", "npg_normalize_input",
    "npg_reconstruct_density", "npg_reconstruct_density_noalloc", "npg_reconstruct_experts", "npg_build_cdf", "npg_sample_dirs", "npg_eval_pdf",
    "npg_mis_alpha", "npg_sample_mis", "npg_eval_pdf_mis", "npg_reconstruct_density5",
    "npg_bin_boundaries", "npg_set_option", "npg_reconstruct_fused", "npg_autotune", "npg_tune_table",
    "npg_serve_create", "npg_serve_destroy", "npg_serve_submit_recon", "npg_serve_submit_sample",
    "npg_serve_poll", "npg_serve_wait", "npg_serve_tables", "npg_serve_copy_tables", "npg_serve_release",
    "npg_serve_get_stats", "npg_serve_last_error",
]


class NpgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"npg error {code}: {msg}")
        self.code = code


class Tables(C.Structure):
    _fields_ = [("pdf_dev", C.c_void_p), ("marg_dev", C.c_void_p), ("cond_dev", C.c_void_p),
                ("total_dev", C.c_void_p), ("L", C.c_uint32), ("H", C.c_int32), ("W", C.c_int32)]


class HierParams(C.Structure):
    _fields_ = [("split_count", C.c_uint32), ("max_depth", C.c_int32)]


class KDGridParams(C.Structure):
    _fields_ = [("res", C.c_int32), ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("split_count", C.c_double),
                ("split_var", C.c_double), ("max_depth", C.c_int32)]


class ServeParams(C.Structure):
    _fields_ = [("n_slots", C.c_uint32), ("max_batch_leaves", C.c_uint32), ("table_bytes", C.c_uint64),
                ("slot_scratch_bytes", C.c_uint64), ("precision", C.c_int)]


class ServeStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "completed", "batches", "leaves", "merged_requests",
                                          "max_concurrent", "queued", "table_bytes_free")]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libnpg.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnpg.so not built at {path}; run python -m paper_2010_01775_amd.build")
    lib = C.CDLL(path)
    P, I, U32, U64, SZ = C.c_void_p, C.c_int, C.c_uint32, C.c_uint64, C.c_size_t
    sig = {
        "npg_create": (I, [C.POINTER(P), I, U64]),
        "npg_destroy": (None, [P]),
        "npg_last_error": (C.c_char_p, [P]),
        "npg_sync_status": (I, [P, P]),
        "npg_memory_usage": (None, [P, C.POINTER(U64), C.POINTER(U64)]),
        "npg_conv_flops": (None, [P, C.POINTER(C.c_double), C.POINTER(C.c_double), I]),
        "npg_model_load": (I, [P, P, SZ, C.POINTER(P)]),
        "npg_model_free": (None, [P]),
        "npg_model_calibrate_fp8": (I, [P, P, P, U32, I, I, P]),
        "npg_build_hierarchy_sorted": (I, [P, P, P, P, U64, C.POINTER(HierParams), P, P, P, P, P, P, U32,
                                           C.POINTER(U32), P]),
        "npg_build_hierarchy": (I, [P, P, U64, C.POINTER(HierParams), P, P, P, P, P, U32,
                                    C.POINTER(U32), P]),
        "npg_mark_valid": (I, [P, C.POINTER(KDGridParams), P, U64, P, P]),
        "npg_build_kdgrid": (I, [P, C.POINTER(KDGridParams), P, P, U64, P, P, P, P, P, U32, C.POINTER(U32),
                                 C.POINTER(U32), P]),
        "npg_locate": (I, [P, C.POINTER(KDGridParams), P, P, U32, P, U64, P, P]),
        "npg_splat_histograms": (I, [P, P, P, P, P, U32, I, I, P, P, I, P]),
        "npg_normalize_input": (I, [P, P, U32, I, I, P, P]),
        "npg_reconstruct_density": (I, [P, P, P, P, U32, I, I, I, P, P]),
        "npg_reconstruct_density_noalloc": (I, [P, P, P, U32, I, I, I, P, P]),
        "npg_reconstruct_experts": (I, [P, P, I, P, P, P, U32, I, I, I, P, P, P]),
        "npg_reconstruct_density5": (I, [P, P, P, P, P, P, U32, I, I, I, P, P]),
        "npg_build_cdf": (I, [P, P, U32, I, I, P, P, P, P, P]),
        "npg_sample_dirs": (I, [P, C.POINTER(Tables), P, P, U64, P, P, P, P]),
        "npg_eval_pdf": (I, [P, C.POINTER(Tables), P, P, U64, P, P]),
        "npg_mis_alpha": (I, [P, P, P, P, P, U32, P, P]),
        "npg_sample_mis": (I, [P, C.POINTER(Tables), P, P, P, P, U64, P, P, P, P]),
        "npg_eval_pdf_mis": (I, [P, C.POINTER(Tables), P, P, P, P, U64, P, P]),
        "npg_bin_boundaries": (I, [I, P]),
        "npg_set_option": (I, [P, C.c_char_p, C.c_int64]),
        "npg_reconstruct_fused": (I, [P, P, P, P, P, P, U32, I, I, I, P, P, P, P, P]),
        "npg_autotune": (I, [P, P, I, I, I, U32, P]),
        "npg_tune_table": (I, [P, P, I, I, I, P, I]),
        "npg_serve_create": (I, [P, P, C.POINTER(ServeParams), C.POINTER(P)]),
        "npg_serve_destroy": (None, [P]),
        "npg_serve_submit_recon": (I, [P, P, P, P, P, U32, I, I, C.POINTER(U64)]),
        "npg_serve_submit_sample": (I, [P, U64, P, P, U64, P, P, C.POINTER(U64)]),
        "npg_serve_poll": (I, [P, U64, C.POINTER(C.c_double)]),
        "npg_serve_wait": (I, [P, U64, C.POINTER(C.c_double)]),
        "npg_serve_tables": (I, [P, U64, C.POINTER(Tables)]),
        "npg_serve_copy_tables": (I, [P, U64, P, P, P, P, P]),
        "npg_serve_release": (I, [P, U64]),
        "npg_serve_get_stats": (None, [P, C.POINTER(ServeStats)]),
        "npg_serve_last_error": (C.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _dev(t, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Context:
    """An npg context on one device with an HBM budget for library scratch."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.npg_create(C.byref(h), device, hbm_budget_bytes)
        if rc:
            raise NpgError(rc, "npg_create failed")
        self.h = h

    def check(self, rc: int):
        if rc:
            raise NpgError(rc, self.lib.npg_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            torch.cuda.synchronize(self.device)
            self.lib.npg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.npg_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_option(self, name: str, value: int):
        self.check(self.lib.npg_set_option(self.h, name.encode(), int(value)))

    def memory_usage(self):
        cur, peak = C.c_uint64(), C.c_uint64()
        self.lib.npg_memory_usage(self.h, C.byref(cur), C.byref(peak))
        return cur.value, peak.value

    def conv_flops(self, reset: bool = False):
        """(matrix-core, vector-ALU) FLOPs of the network convolutions launched
        since the last reset, as each layer was launched."""
        mat, vec = C.c_double(), C.c_double()
        self.lib.npg_conv_flops(self.h, C.byref(mat), C.byref(vec), int(bool(reset)))
        return mat.value, vec.value


def sync_status(ctx: Context, stream=None) -> int:
    """Synchronise and return the data-dependent error status (0 or E_RANGE)."""
    return ctx.lib.npg_sync_status(ctx.h, _stream(stream))


class Model:
    def __init__(self, ctx: Context, weight_file: bytes):
        self.ctx = ctx
        buf = C.create_string_buffer(weight_file, len(weight_file))
        h = C.c_void_p()
        ctx.check(ctx.lib.npg_model_load(ctx.h, buf, len(weight_file), C.byref(h)))
        self.h = h

    def calibrate_fp8(self, energy, stream=None):
        L, H, W = energy.shape
        self.ctx.check(self.ctx.lib.npg_model_calibrate_fp8(self.ctx.h, self.h, _ptr(energy), L, H, W,
                                                            _stream(stream)))

    def free(self):
        if getattr(self, "h", None):
            self.ctx.lib.npg_model_free(self.h)
            self.h = None


def model_load(ctx: Context, weight_file: bytes) -> Model:
    return Model(ctx, weight_file)


@dataclass
class CdfTables:
    pdf: torch.Tensor
    marg: torch.Tensor
    cond: torch.Tensor
    total: torch.Tensor

    def c(self) -> Tables:
        L, H, W = self.pdf.shape
        return Tables(self.pdf.data_ptr(), self.marg.data_ptr(), self.cond.data_ptr(),
                      self.total.data_ptr() if self.total is not None else None, L, H, W)


def build_hierarchy_sorted(ctx: Context, pos, dirs, w, split_count: int = 8192, max_depth: int = 6,
                           max_leaves: int | None = None, out=None, stream=None):
    """build_hierarchy plus the photons' directions and weights in leaf order
    (dirs_sorted[i] = dirs[perm[i]], w_sorted[i] = w[perm[i]]).  out: optional
    dict of caller tensors perm, dirs, w, leaf_off to write into."""
    _dev(pos, torch.float32, "pos")
    _dev(dirs, torch.float32, "dirs")
    _dev(w, torch.int32, "w (uint32 bits in int32)")
    n = pos.shape[0]
    if dirs.shape != (n, 3) or w.shape != (n,):
        raise ValueError("dirs must be [n][3] and w [n]")
    dev = pos.device
    if max_leaves is None:
        max_leaves = max(1, min(n, 8 ** max_depth))
    out = out or {}
    perm = out.get("perm", torch.empty(n, dtype=torch.int32, device=dev))
    ds = out.get("dirs", torch.empty((n, 3), dtype=torch.float32, device=dev))
    ws = out.get("w", torch.empty(n, dtype=torch.int32, device=dev))
    off = out.get("leaf_off", torch.empty(max_leaves + 1, dtype=torch.int32, device=dev))
    key = torch.empty(max_leaves, dtype=torch.int64, device=dev)
    depth = torch.empty(max_leaves, dtype=torch.uint8, device=dev)
    nl = C.c_uint32(0)
    prm = HierParams(split_count, max_depth)
    rc = ctx.lib.npg_build_hierarchy_sorted(ctx.h, _ptr(pos), _ptr(dirs), _ptr(w), n, C.byref(prm), _ptr(perm),
                                            _ptr(ds), _ptr(ws), _ptr(off), _ptr(key), _ptr(depth), max_leaves,
                                            C.byref(nl), _stream(stream))
    ctx.check(rc)
    L = nl.value
    return dict(perm=perm, dirs=ds, w=ws, leaf_off=off[:L + 1], key=key[:L], depth=depth[:L], n_leaves=L)


def build_hierarchy(ctx: Context, pos, split_count: int = 8192, max_depth: int = 6,
                    max_leaves: int | None = None, want_leaf_of: bool = True, stream=None,
                    leaf_of_out=None):
    """Octree leaves of the photon positions; returns a dict of device tensors.
    leaf_of_out: optional caller tensor (int32 [n]) for the per-photon leaf ids."""
    _dev(pos, torch.float32, "pos")
    n = pos.shape[0]
    dev = pos.device
    if max_leaves is None:
        max_leaves = max(1, min(n, 8 ** max_depth))
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    if leaf_of_out is not None:
        _dev(leaf_of_out, torch.int32, "leaf_of_out")
        if leaf_of_out.shape != (n,):
            raise ValueError("leaf_of_out must have shape (n,)")
        leaf_of = leaf_of_out
    else:
        leaf_of = torch.empty(n, dtype=torch.int32, device=dev) if want_leaf_of else None
    off = torch.empty(max_leaves + 1, dtype=torch.int32, device=dev)
    key = torch.empty(max_leaves, dtype=torch.int64, device=dev)
    depth = torch.empty(max_leaves, dtype=torch.uint8, device=dev)
    nl = C.c_uint32(0)
    prm = HierParams(split_count, max_depth)
    rc = ctx.lib.npg_build_hierarchy(ctx.h, _ptr(pos), n, C.byref(prm), _ptr(perm), _ptr(leaf_of),
                                     _ptr(off), _ptr(key), _ptr(depth), max_leaves, C.byref(nl),
                                     _stream(stream))
    ctx.check(rc)
    L = nl.value
    return dict(perm=perm, leaf_of=leaf_of, leaf_off=off[:L + 1], key=key[:L], depth=depth[:L],
                n_leaves=L)


# the paper's grid: 100^3 voxels, split while the count exceeds 500 * sqrt(2^t)
# at iteration t or the normal variance exceeds 0.5, local trees of depth <= 8
PAPER_GRID_RES = 100
PAPER_SPLIT_VAR = 0.5
PAPER_MAX_DEPTH = 8


def paper_split_count(t: int, c: float = 500.0) -> float:
    return c * math.sqrt(2.0 ** t)


def kdgrid_params(res=PAPER_GRID_RES, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), split_count=None,
                  split_var=PAPER_SPLIT_VAR, max_depth=PAPER_MAX_DEPTH) -> KDGridParams:
    sc = paper_split_count(1) if split_count is None else float(split_count)
    return KDGridParams(int(res), (C.c_float * 3)(*lo), (C.c_float * 3)(*hi), sc, float(split_var), int(max_depth))


def mark_valid(ctx: Context, params: KDGridParams, pts, valid=None, stream=None):
    """uint8 [res^3] mask of the voxels holding at least one point."""
    _dev(pts, torch.float32, "pts")
    if valid is None:
        valid = torch.empty(params.res ** 3, dtype=torch.uint8, device=pts.device)
    ctx.check(ctx.lib.npg_mark_valid(ctx.h, C.byref(params), _ptr(pts), pts.shape[0], _ptr(valid), _stream(stream)))
    return valid


def build_kdgrid(ctx: Context, params: KDGridParams, pos, normal=None, valid=None, max_leaves: int | None = None,
                 stream=None, out=None):
    """The hierarchical grid over the photons; returns a dict of device
    tensors (perm, leaf_off, cell_root, nodes as int32 pairs) and counts.
    out: optional dict of preallocated perm / leaf_off / cell_root / nodes."""
    _dev(pos, torch.float32, "pos")
    n = pos.shape[0]
    dev = pos.device
    if normal is not None:
        _dev(normal, torch.float32, "normal")
    if valid is not None:
        _dev(valid, torch.uint8, "valid")
    if max_leaves is None:
        max_leaves = max(1, min(n, (1 << 29) - 1))
    nv = params.res ** 3
    o = out or {}
    perm = o.get("perm") if o.get("perm") is not None else torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    off = o.get("leaf_off") if o.get("leaf_off") is not None else torch.empty(max_leaves + 1, dtype=torch.int32,
                                                                             device=dev)
    root = o.get("cell_root") if o.get("cell_root") is not None else torch.empty(nv, dtype=torch.int32, device=dev)
    nodes = o.get("nodes") if o.get("nodes") is not None else torch.empty((2 * max_leaves, 2), dtype=torch.int32,
                                                                           device=dev)
    nl, nn = C.c_uint32(0), C.c_uint32(0)
    ctx.check(ctx.lib.npg_build_kdgrid(ctx.h, C.byref(params), _ptr(pos), _ptr(normal), n, _ptr(valid), _ptr(perm),
                                       _ptr(off), _ptr(root), _ptr(nodes), max_leaves, C.byref(nl), C.byref(nn),
                                       _stream(stream)))
    L = nl.value
    return dict(perm=perm, leaf_off=off[:L + 1], cell_root=root, nodes=nodes[:nn.value], n_leaves=L,
                n_nodes=nn.value)


def locate(ctx: Context, params: KDGridParams, grid: dict, q, out=None, stream=None):
    """Leaf id (uint32 bits in int32; -1 = none) of each query point."""
    _dev(q, torch.float32, "q")
    if out is None:
        out = torch.empty(q.shape[0], dtype=torch.int32, device=q.device)
    ctx.check(ctx.lib.npg_locate(ctx.h, C.byref(params), _ptr(grid["cell_root"]), _ptr(grid["nodes"]),
                                 grid["n_nodes"], _ptr(q), q.shape[0], _ptr(out), _stream(stream)))
    return out


def splat_histograms(ctx: Context, dirs, w, leaf_off, H: int, W: int, perm=None, energy=None,
                     count=None, accumulate: bool = False, want_count: bool = True, stream=None):
    _dev(dirs, torch.float32, "dirs")
    _dev(w, torch.int32, "w (uint32 bits in int32)")
    _dev(leaf_off, torch.int32, "leaf_off")
    L = leaf_off.shape[0] - 1
    dev = dirs.device
    if energy is None:
        energy = torch.empty((L, H, W), dtype=torch.int64, device=dev)
    if count is None and want_count:
        count = torch.empty((L, H, W), dtype=torch.int32, device=dev)
    ctx.check(ctx.lib.npg_splat_histograms(ctx.h, _ptr(dirs), _ptr(w), _ptr(perm), _ptr(leaf_off), L,
                                           H, W, _ptr(energy), _ptr(count), int(bool(accumulate)),
                                           _stream(stream)))
    return energy, count


def normalize_input(ctx: Context, energy, x=None, stream=None):
    L, H, W = energy.shape
    if x is None:
        x = torch.empty((L, H, W), dtype=torch.float32, device=energy.device)
    ctx.check(ctx.lib.npg_normalize_input(ctx.h, _ptr(energy), L, H, W, _ptr(x), _stream(stream)))
    return x


def reconstruct_density(ctx: Context, model: Model, energy, precision="fp32", count=None,
                        density=None, stream=None):
    L, H, W = energy.shape
    if density is None:
        density = torch.empty((L, H, W), dtype=torch.float32, device=energy.device)
    p = PRECISION[precision] if isinstance(precision, str) else int(precision)
    ctx.check(ctx.lib.npg_reconstruct_density(ctx.h, model.h, _ptr(energy), _ptr(count), L, H, W, p,
                                              _ptr(density), _stream(stream)))
    return density


def reconstruct_density_noalloc(ctx: Context, model: Model, energy, precision="fp32", density=None, stream=None):
    """reconstruct_density through the library's static scratch array: the
    call allocates no device memory (pass `density` to keep it so)."""
    L, H, W = energy.shape
    if density is None:
        density = torch.empty((L, H, W), dtype=torch.float32, device=energy.device)
    p = PRECISION[precision] if isinstance(precision, str) else int(precision)
    ctx.check(ctx.lib.npg_reconstruct_density_noalloc(ctx.h, model.h, _ptr(energy), L, H, W, p, _ptr(density),
                                                      _stream(stream)))
    return density


def reconstruct_density5(ctx: Context, model: Model, energy, count, energy_prev, count_prev, precision="fp32",
                         density=None, stream=None):
    """Densities from the paper's five input channels (maps and photon counts
    of iterations t and t-1, valid-bin mask)."""
    L, H, W = energy.shape
    for t, name in ((energy, "energy"), (energy_prev, "energy_prev")):
        _dev(t, torch.int64, f"{name} (uint64 bits in int64)")
        if t.shape != (L, H, W):
            raise ValueError(f"{name} must be [L][H][W]")
    for t, name in ((count, "count"), (count_prev, "count_prev")):
        _dev(t, torch.int32, f"{name} (uint32 bits in int32)")
        if t.shape != (L, H, W):
            raise ValueError(f"{name} must be [L][H][W]")
    if density is None:
        density = torch.empty((L, H, W), dtype=torch.float32, device=energy.device)
    p = PRECISION[precision] if isinstance(precision, str) else int(precision)
    ctx.check(ctx.lib.npg_reconstruct_density5(ctx.h, model.h, _ptr(energy), _ptr(count), _ptr(energy_prev),
                                               _ptr(count_prev), L, H, W, p, _ptr(density), _stream(stream)))
    return density


# photon-count ranges of the five experts: [0,100), [100,500), [500,1000),
# [1000,5000), [5000,inf)
PAPER_EXPERT_BOUNDS = (100, 500, 1000, 5000)


def reconstruct_experts(ctx: Context, models, leaf_off, energy, precision="fp32",
                        bounds=PAPER_EXPERT_BOUNDS, density=None, stream=None):
    """Densities with one model per photon-count range; returns
    (density, leaves per expert)."""
    _dev(leaf_off, torch.int32, "leaf_off")
    L, H, W = energy.shape
    if leaf_off.shape != (L + 1,):
        raise ValueError("leaf_off must have L + 1 entries")
    if density is None:
        density = torch.empty((L, H, W), dtype=torch.float32, device=energy.device)
    n = len(models)
    hs = (C.c_void_p * n)(*[m.h for m in models])
    bd = (C.c_uint32 * max(1, len(bounds)))(*bounds)
    counts = (C.c_uint32 * n)()
    p = PRECISION[precision] if isinstance(precision, str) else int(precision)
    ctx.check(ctx.lib.npg_reconstruct_experts(ctx.h, hs, n, bd, _ptr(leaf_off), _ptr(energy), L, H, W, p,
                                              _ptr(density), counts, _stream(stream)))
    return density, list(counts)


def _new_tables(L, H, W, dev):
    return CdfTables(torch.empty((L, H, W), dtype=torch.float32, device=dev),
                     torch.empty((L, H + 1), dtype=torch.float32, device=dev),
                     torch.empty((L, H, W + 1), dtype=torch.float32, device=dev),
                     torch.empty(L, dtype=torch.float64, device=dev))


def reconstruct_fused(ctx: Context, model: Model, dirs, w, leaf_off, H: int, W: int, precision="fp32",
                      perm=None, out: CdfTables | None = None, stream=None) -> CdfTables:
    """splat -> normalise -> network -> CDF in one call (chunked, scratch-resident maps)."""
    L = leaf_off.shape[0] - 1
    if out is None:
        out = _new_tables(L, H, W, dirs.device)
    p = PRECISION[precision] if isinstance(precision, str) else int(precision)
    ctx.check(ctx.lib.npg_reconstruct_fused(ctx.h, model.h, _ptr(dirs), _ptr(w), _ptr(perm), _ptr(leaf_off), L,
                                            H, W, p, _ptr(out.pdf), _ptr(out.marg), _ptr(out.cond),
                                            _ptr(out.total), _stream(stream)))
    return out


def autotune(ctx: Context, model: Model, H: int, W: int, precision="fp32", probe_leaves: int = 1024,
             stream=None):
    p = PRECISION[precision] if isinstance(precision, str) else int(precision)
    ctx.check(ctx.lib.npg_autotune(ctx.h, model.h, H, W, p, probe_leaves, _stream(stream)))
    return tune_table(ctx, model, H, W, precision)


def tune_table(ctx: Context, model: Model, H: int, W: int, precision="fp32"):
    import numpy as np
    p = PRECISION[precision] if isinstance(precision, str) else int(precision)
    buf = np.zeros(256, np.int32)
    n = ctx.lib.npg_tune_table(ctx.h, model.h, H, W, p, buf.ctypes.data, 256)
    return [int(v) for v in buf[:n]]


def build_cdf(ctx: Context, density, out: CdfTables | None = None, stream=None) -> CdfTables:
    L, H, W = density.shape
    dev = density.device
    if out is None:
        out = _new_tables(L, H, W, dev)
    ctx.check(ctx.lib.npg_build_cdf(ctx.h, _ptr(density), L, H, W, _ptr(out.pdf), _ptr(out.marg),
                                    _ptr(out.cond), _ptr(out.total), _stream(stream)))
    return out


def sample_dirs(ctx: Context, tables: CdfTables, leaf, u, want_bin: bool = True, out=None,
                stream=None):
    n = leaf.shape[0]
    dev = leaf.device
    if out is None:
        out = (torch.empty((n, 3), dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.int32, device=dev) if want_bin else None)
    d, p, b = out
    t = tables.c()
    ctx.check(ctx.lib.npg_sample_dirs(ctx.h, C.byref(t), _ptr(leaf), _ptr(u), n, _ptr(d), _ptr(p),
                                      _ptr(b), _stream(stream)))
    return d, p, b


def eval_pdf(ctx: Context, tables: CdfTables, leaf, dirs, out=None, stream=None):
    n = leaf.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=leaf.device)
    t = tables.c()
    ctx.check(ctx.lib.npg_eval_pdf(ctx.h, C.byref(t), _ptr(leaf), _ptr(dirs), n, _ptr(out),
                                   _stream(stream)))
    return out


def mis_alpha(ctx: Context, nu_b, nu_g, q_b, q_g, out=None, stream=None):
    """Per-leaf one-sample MIS weight from the path statistics."""
    _dev(nu_b, torch.float32, "nu_b")
    _dev(nu_g, torch.float32, "nu_g")
    _dev(q_b, torch.int32, "q_b (uint32 bits in int32)")
    _dev(q_g, torch.int32, "q_g (uint32 bits in int32)")
    L = nu_b.shape[0]
    if out is None:
        out = torch.empty(L, dtype=torch.float32, device=nu_b.device)
    ctx.check(ctx.lib.npg_mis_alpha(ctx.h, _ptr(nu_b), _ptr(nu_g), _ptr(q_b), _ptr(q_g), L, _ptr(out),
                                    _stream(stream)))
    return out


def sample_mis(ctx: Context, tables: CdfTables, alpha, leaf, normal, u, out=None, stream=None):
    """One-sample MIS directions; returns (dirs, pdf, strategy: 1 = BSDF)."""
    n = leaf.shape[0]
    dev = leaf.device
    if out is None:
        out = (torch.empty((n, 3), dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.float32, device=dev),
               torch.empty(n, dtype=torch.uint8, device=dev))
    d, p, st = out
    t = tables.c()
    ctx.check(ctx.lib.npg_sample_mis(ctx.h, C.byref(t), _ptr(alpha), _ptr(leaf), _ptr(normal), _ptr(u), n,
                                     _ptr(d), _ptr(p), _ptr(st), _stream(stream)))
    return d, p, st


def eval_pdf_mis(ctx: Context, tables: CdfTables, alpha, leaf, normal, dirs, out=None, stream=None):
    n = leaf.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=leaf.device)
    t = tables.c()
    ctx.check(ctx.lib.npg_eval_pdf_mis(ctx.h, C.byref(t), _ptr(alpha), _ptr(leaf), _ptr(normal), _ptr(dirs), n,
                                       _ptr(out), _stream(stream)))
    return out


def bin_boundaries(W: int):
    import numpy as np
    out = np.empty(2 * W, np.float32)
    rc = load_library().npg_bin_boundaries(W, out.ctypes.data)
    if rc:
        raise NpgError(rc, "bad W")
    return out.reshape(W, 2)


class Server:
    """Continuous-batching server over one context's device (see npg.h)."""

    def __init__(self, ctx: Context, model: Model, n_slots: int = 4, max_batch_leaves: int = 8192,
                 table_bytes: int = 8 << 30, slot_scratch_bytes: int = 2 << 30, precision="bf16"):
        import numpy as np  # noqa: F401
        self.ctx, self.model = ctx, model
        p = PRECISION[precision] if isinstance(precision, str) else int(precision)
        prm = ServeParams(n_slots, max_batch_leaves, table_bytes, slot_scratch_bytes, p)
        h = C.c_void_p()
        ctx.check(ctx.lib.npg_serve_create(ctx.h, model.h, C.byref(prm), C.byref(h)))
        self.h = h
        self.lib = ctx.lib

    def _raise(self, rc, what):
        raise NpgError(rc, f"{what}: {self.lib.npg_serve_last_error(self.h).decode()}")

    def submit_recon(self, dirs, w, begin, count, H: int, W: int) -> int:
        import numpy as np
        b = np.ascontiguousarray(begin, dtype=np.uint32)
        c = np.ascontiguousarray(count, dtype=np.uint32)
        t = C.c_uint64()
        self.ctx.check(self.lib.npg_serve_submit_recon(self.h, _ptr(dirs), _ptr(w), b.ctypes.data, c.ctypes.data,
                                                        len(b), H, W, C.byref(t)))
        return t.value

    def submit_sample(self, recon: int, leaf, u, dir_out, pdf_out) -> int:
        t = C.c_uint64()
        self.ctx.check(self.lib.npg_serve_submit_sample(self.h, recon, _ptr(leaf), _ptr(u), leaf.shape[0],
                                                         _ptr(dir_out), _ptr(pdf_out), C.byref(t)))
        return t.value

    def poll(self, ticket: int):
        lat = C.c_double()
        rc = self.lib.npg_serve_poll(self.h, ticket, C.byref(lat))
        if rc < 0:
            self._raise(rc, "request failed")
        return (lat.value if rc == 1 else None)

    def wait(self, ticket: int) -> float:
        lat = C.c_double()
        rc = self.lib.npg_serve_wait(self.h, ticket, C.byref(lat))
        if rc < 0:
            self._raise(rc, "request failed")
        return lat.value

    def copy_tables(self, ticket: int, out: CdfTables, stream=None):
        rc = self.lib.npg_serve_copy_tables(self.h, ticket, _ptr(out.pdf), _ptr(out.marg), _ptr(out.cond),
                                            _ptr(out.total), _stream(stream))
        if rc:
            self._raise(rc, "copy_tables failed")
        return out

    def release(self, ticket: int):
        rc = self.lib.npg_serve_release(self.h, ticket)
        if rc:
            self._raise(rc, "release failed")

    def stats(self) -> dict:
        st = ServeStats()
        self.lib.npg_serve_get_stats(self.h, C.byref(st))
        return {n: getattr(st, n) for n, _ in ServeStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.npg_serve_destroy(self.h)
            self.h = None
