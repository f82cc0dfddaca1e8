// The paper's hierarchical grid: a regular grid of res^3 voxels, valid
// voxels marked by camera-path bounce points, and every valid voxel split
// into a local binary KD tree (Sec. 7.1 "Voxel subdivision"; Sec. 8,
// path-guiding details).
//
// Build, level by level (every node of a level is independent):
//   1. voxel id of each photon (FP64 rule; invalid voxels get a sentinel
//      key), stable radix sort of (voxel, photon index): the photons of a
//      voxel become one contiguous segment, in ascending photon index;
//   2. segment starts = the roots, in ascending voxel id;
//   3. per level: the split test of each node (count, and the normal
//      variance from exact integer sums) and, for a splitting node, the
//      median coordinate on the longest axis by an exact radix select over
//      its segment (8 bits per pass from the highest bit where the node's
//      keys differ), one wavefront per node of up to 2048 photons and one
//      workgroup per larger node; then a stable partition of each
//      splitting node's segment into its two child segments, in place
//      (child slots from a scan of the split flags, so node ids do not
//      depend on scheduling); a node that does not split keeps its segment
//      where it is and becomes a leaf;
//   4. leaves sorted by segment start: depth-first order inside a voxel,
//      voxels ascending, since every split keeps its children inside the
//      parent's segment, first child first.
// Point location: voxel id, then down the tree by the split comparisons.
#include "npg_internal.h"

namespace {

constexpr int KD_THREADS = 256;
constexpr uint32_t KD_NONE = 0xFFFFFFFFu;
constexpr double KD_QSCALE = 1048576.0;  // normals quantised to multiples of 2^-20

struct GridDev {
  int res;
  float lo[3];
  double invr[3];  // res / (hi - lo)
  double step[3];  // (hi - lo) / res
};

// Monotone map of float32 to uint32 (-0 read as +0): a < b iff key(a) < key(b).
__device__ __forceinline__ uint32_t okey(float x) {
  const uint32_t b = __float_as_uint(x == 0.0f ? 0.0f : x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float okey_inv(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Voxel coordinate on one axis: floor((p - lo) * invr) in FP64 (no
// contraction), clamped to [0, res-1].
__device__ __forceinline__ int vox_axis(float p, float lo, double invr, int res) {
  const double t = __dmul_rn(__dsub_rn((double)p, (double)lo), invr);
  const double f = floor(t);
  return f < 0.0 ? 0 : (f > (double)(res - 1) ? res - 1 : (int)f);
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
  return isfinite(x) && isfinite(y) && isfinite(z);
}

__device__ __forceinline__ uint32_t vox_id(const GridDev &g, float x, float y, float z) {
  const uint32_t r = (uint32_t)g.res;
  return (uint32_t)vox_axis(x, g.lo[0], g.invr[0], g.res) +
         r * ((uint32_t)vox_axis(y, g.lo[1], g.invr[1], g.res) + r * (uint32_t)vox_axis(z, g.lo[2], g.invr[2], g.res));
}

__global__ __launch_bounds__(256) void kd_mark_kernel(GridDev g, const float *__restrict__ p, uint64_t n,
                                                      uint8_t *__restrict__ valid, uint32_t *err) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
    if (!finite3(x, y, z)) {
      raise_err(err, ERR_RANGE);
      continue;
    }
    valid[vox_id(g, x, y, z)] = 1;
  }
}

// key = voxel id, or `sent` (sorts last) for an invalid voxel or a bad
// position; a non-finite position, or normal of a photon in a valid voxel,
// raises the range error
__global__ __launch_bounds__(256) void kd_keys_kernel(GridDev g, const float *__restrict__ p,
                                                      const float *__restrict__ nrm, uint64_t n,
                                                      const uint8_t *__restrict__ valid, uint32_t sent,
                                                      uint32_t *__restrict__ key, uint32_t *err) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
    uint32_t k = sent;
    if (!finite3(x, y, z)) {
      raise_err(err, ERR_RANGE);
    } else {
      const uint32_t v = vox_id(g, x, y, z);
      if (!valid || valid[v]) {
        k = v;
        if (nrm && !finite3(nrm[3 * i], nrm[3 * i + 1], nrm[3 * i + 2])) raise_err(err, ERR_RANGE);
      }
    }
    key[i] = k;
  }
}

// flag[i] = 1 at the first photon of each valid voxel's segment; *nvalid =
// number of photons in valid voxels (the sentinel keys sort last)
__global__ __launch_bounds__(256) void kd_seg_kernel(const uint32_t *__restrict__ ks, uint64_t n, uint32_t sent,
                                                     uint32_t *__restrict__ flag, uint32_t *nvalid) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t k = ks[i];
    flag[i] = (k != sent && (i == 0 || ks[i - 1] != k)) ? 1u : 0u;
    if (k != sent && (i + 1 == n || ks[i + 1] == sent)) *nvalid = (uint32_t)(i + 1);
  }
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t *__restrict__ a, uint64_t n, int32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Per-level node records (structure of arrays).
struct Level {
  uint32_t *start, *count, *id;
  double *box;  // [6] per node: lo xyz, hi xyz
};

// roots: node j = j-th valid non-empty voxel
__global__ __launch_bounds__(256) void kd_roots_kernel(GridDev g, const uint32_t *__restrict__ ks,
                                                       const uint32_t *__restrict__ flag,
                                                       const uint32_t *__restrict__ seg, uint64_t n,
                                                       Level lv, int32_t *__restrict__ cell_root) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    const uint32_t j = seg[i], v = ks[i];
    lv.start[j] = (uint32_t)i;
    lv.id[j] = j;
    cell_root[v] = (int32_t)j;
    const uint32_t r = (uint32_t)g.res;
    const uint32_t c[3] = {v % r, (v / r) % r, v / (r * r)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lv.box[6 * (size_t)j + a] = __dadd_rn((double)g.lo[a], __dmul_rn((double)c[a], g.step[a]));
      lv.box[6 * (size_t)j + 3 + a] = __dadd_rn((double)g.lo[a], __dmul_rn((double)(c[a] + 1), g.step[a]));
    }
  }
}

__global__ __launch_bounds__(256) void kd_root_counts_kernel(Level lv, uint32_t n0, const uint32_t *nvalid) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n0) lv.count[j] = (j + 1 < n0 ? lv.start[j + 1] : *nvalid) - lv.start[j];
}

// Workgroup-wide sums of three int64 values (exact, so the order is free).
__device__ __forceinline__ void wg_sum3_i64(long long v[3], long long (*red)[KD_THREADS / 64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[a] += __shfl_xor(v[a], o);
    if (lane == 0) red[a][wave] = v[a];
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    long long t = 0;
#pragma unroll
    for (int w = 0; w < KD_THREADS / 64; ++w) t += red[a][w];
    v[a] = t;
  }
}

// Split test of one node from its photons' normals: V > split_var, with V
// from exact integer sums (the order of the sums does not matter).
__device__ __forceinline__ bool variance_exceeds(long long sx_, long long sy_, long long sz_, uint32_t M,
                                                 double split_var) {
  const double sx = (double)sx_, sy = (double)sy_, sz = (double)sz_;
  const double num = __dadd_rn(__dadd_rn(__dmul_rn(sx, sx), __dmul_rn(sy, sy)), __dmul_rn(sz, sz));
  const double den = __dmul_rn(__dmul_rn((double)M, (double)M), KD_QSCALE * KD_QSCALE);
  return __dsub_rn(1.0, __ddiv_rn(num, den)) > split_var;
}

// One photon's quantised normal added to s[3]; a non-finite component counts
// as 0 and sets *bad.
__device__ __forceinline__ void add_qnormal(const float *__restrict__ nrm, uint32_t ph, long long s[3], bool *bad) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float v = nrm[3 * (size_t)ph + a];
    if (!isfinite(v)) *bad = true;
    const double c = isfinite(v) ? fmin(fmax((double)v, -1.0), 1.0) : 0.0;
    s[a] += (long long)rint(c * KD_QSCALE);
  }
}

// Longest axis of a node's box (ties: the lower axis).
__device__ __forceinline__ uint32_t longest_axis(const double *b) {
  double ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) ext[a] = __dsub_rn(b[3 + a], b[a]);
  uint32_t axis = 0;
  if (ext[1] > ext[axis]) axis = 1;
  if (ext[2] > ext[axis]) axis = 2;
  return axis;
}

// Nodes of more than KD_WAVE_MAX photons take a whole workgroup; smaller ones
// one wavefront each.
constexpr uint32_t KD_WAVE_MAX = 2048;

// Split test and median selection, one workgroup per node of a list (the
// nodes above KD_WAVE_MAX photons; grid-stride over the list, whose length
// the wavefront kernel wrote to *nbig).  Outputs per node: sflag (1: splits),
// axis, the split key and the number of photons below it.  tkey receives the
// node's photon keys on the split axis (aligned with perm) for the partition.
__global__ __launch_bounds__(KD_THREADS) void kd_select_kernel(const float *__restrict__ pos,
                                                               const float *__restrict__ nrm,
                                                               const uint32_t *__restrict__ perm, Level lv,
                                                               const uint32_t *__restrict__ big,
                                                               const uint32_t *nbig, int depth, int max_depth,
                                                               double split_count, double split_var,
                                                               uint32_t *__restrict__ tkey,
                                                               uint32_t *__restrict__ sflag,
                                                               uint32_t *__restrict__ sel, uint32_t *err) {
  __shared__ long long red[3][KD_THREADS / 64];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wsum[KD_THREADS / 64];
  __shared__ uint32_t pick[2];
  const uint32_t nb = *nbig;
  for (uint32_t bi = blockIdx.x; bi < nb; bi += gridDim.x) {
  __syncthreads();  // shared arrays of the previous node are no longer read
  const uint32_t j = big[bi];
  const uint32_t start = lv.start[j], M = lv.count[j];
  bool split = false;
  if (depth < max_depth && M >= 2) {
    split = (double)M > split_count;
    if (!split && nrm) {
      long long s[3] = {0, 0, 0};
      bool bad = false;
      for (uint32_t i = threadIdx.x; i < M; i += KD_THREADS) add_qnormal(nrm, perm[start + i], s, &bad);
      if (bad) raise_err(err, ERR_RANGE);
      wg_sum3_i64(s, red);
      split = variance_exceeds(s[0], s[1], s[2], M, split_var);
    }
  }
  uint32_t axis = 0, key = 0, less = 0;
  if (split) {
    axis = longest_axis(lv.box + 6 * (size_t)j);
    // exact selection of the (M/2)-th smallest key, 8 bits per pass
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // keys of the split axis, and their range: bits above the highest one
    // where min and max differ are common to every key (and to the median)
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0;
    for (uint32_t i = threadIdx.x; i < M; i += KD_THREADS) {
      const uint32_t k = okey(pos[3 * (size_t)perm[start + i] + axis]);
      tkey[start + i] = k;
      kmin = min(kmin, k);
      kmax = max(kmax, k);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      kmin = min(kmin, (uint32_t)__shfl_xor(kmin, o));
      kmax = max(kmax, (uint32_t)__shfl_xor(kmax, o));
    }
    if (lane == 0) {
      wsum[wave] = kmin;
      hist[wave] = kmax;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < KD_THREADS / 64; ++w) {
      kmin = min(kmin, wsum[w]);
      kmax = max(kmax, hist[w]);
    }
    __syncthreads();
    // exact selection of the (M/2)-th smallest key, 8 bits per pass from the
    // highest differing bit down
    uint32_t m = M / 2;
    const int h = kmin == kmax ? -1 : 31 - __clz(kmin ^ kmax);
    uint32_t pmask = h < 0 ? 0xFFFFFFFFu : (h >= 31 ? 0u : ~((2u << h) - 1u));
    uint32_t prefix = kmin & pmask;
    for (int hi = h; hi >= 0; hi -= 8) {
      const int sh = hi >= 7 ? hi - 7 : 0;
      const uint32_t dmask = (2u << (hi - sh)) - 1u;
      hist[threadIdx.x] = 0;
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < M; i += KD_THREADS) {
        const uint32_t k = tkey[start + i];
        if (((k ^ prefix) & pmask) == 0) atomicAdd(&hist[(k >> sh) & dmask], 1u);
      }
      __syncthreads();
      // inclusive scan of the 256 digit counts (one per thread)
      const uint32_t c = hist[threadIdx.x];
      uint32_t inc = c;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
      }
      if (lane == 63) wsum[wave] = inc;
      __syncthreads();
      for (int w = 0; w < wave; ++w) inc += wsum[w];
      const uint32_t exc = inc - c;
      if (exc <= m && m < inc) {  // exactly one digit holds rank m
        pick[0] = threadIdx.x;
        pick[1] = exc;
      }
      __syncthreads();
      const uint32_t d = pick[0], below = pick[1];
      m -= below;
      less += below;
      prefix |= d << sh;
      pmask |= dmask << sh;
      __syncthreads();
    }
    key = prefix;  // all keys equal (h < 0): the common key, nothing below it
    split = less > 0;
  }
  if (threadIdx.x == 0) {
    sflag[j] = split ? 1u : 0u;
    sel[3 * (size_t)j] = axis;
    sel[3 * (size_t)j + 1] = key;
    sel[3 * (size_t)j + 2] = less;
  }
  }
}

// Orders this wavefront's LDS accesses before and after it (the lanes of a
// wavefront read what other lanes wrote).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The same split test and selection with one wavefront per node (four nodes
// per workgroup) for nodes of at most KD_WAVE_MAX photons; a larger node is
// appended to the list `big` for kd_select_kernel.  Each wavefront works
// alone (its own LDS histogram, no workgroup barrier).
__global__ __launch_bounds__(KD_THREADS) void kd_select_wave_kernel(
    const float *__restrict__ pos, const float *__restrict__ nrm, const uint32_t *__restrict__ perm, Level lv,
    uint32_t active, int depth, int max_depth, double split_count, double split_var, uint32_t *__restrict__ tkey,
    uint32_t *__restrict__ sflag, uint32_t *__restrict__ sel, uint32_t *__restrict__ big, uint32_t *nbig,
    uint32_t *err) {
  __shared__ uint32_t hist_all[KD_THREADS / 64][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t j = blockIdx.x * (KD_THREADS / 64) + wave;
  if (j >= active) return;
  const uint32_t start = lv.start[j], M = lv.count[j];
  if (M > KD_WAVE_MAX) {
    if (lane == 0) big[atomicAdd(nbig, 1u)] = j;
    return;
  }
  uint32_t *hist = hist_all[wave];
  bool split = false;
  if (depth < max_depth && M >= 2) {
    split = (double)M > split_count;
    if (!split && nrm) {
      long long s[3] = {0, 0, 0};
      bool bad = false;
      for (uint32_t i0 = 0; i0 < M; i0 += 4 * 64) {  // four photons in flight per lane
        uint32_t ph[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t i = i0 + 64 * q + lane;
          ph[q] = i < M ? perm[start + i] : KD_NONE;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (ph[q] != KD_NONE) add_qnormal(nrm, ph[q], s, &bad);
      }
      if (bad) raise_err(err, ERR_RANGE);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s[a] += __shfl_xor(s[a], o);
      split = variance_exceeds(s[0], s[1], s[2], M, split_var);
    }
  }
  uint32_t axis = 0, key = 0, less = 0;
  if (split) {
    axis = longest_axis(lv.box + 6 * (size_t)j);
    // keys of the split axis and their range (as in kd_select_kernel)
    uint32_t kmin = 0xFFFFFFFFu, kmax = 0;
    for (uint32_t i0 = 0; i0 < M; i0 += 4 * 64) {  // four keys in flight per lane
      uint32_t ph[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = i0 + 64 * q + lane;
        ph[q] = i < M ? perm[start + i] : KD_NONE;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (ph[q] == KD_NONE) continue;
        const uint32_t k = okey(pos[3 * (size_t)ph[q] + axis]);
        tkey[start + i0 + 64 * q + lane] = k;
        kmin = min(kmin, k);
        kmax = max(kmax, k);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      kmin = min(kmin, (uint32_t)__shfl_xor(kmin, o));
      kmax = max(kmax, (uint32_t)__shfl_xor(kmax, o));
    }
    uint32_t m = M / 2;
    const int h = kmin == kmax ? -1 : 31 - __clz(kmin ^ kmax);
    uint32_t pmask = h < 0 ? 0xFFFFFFFFu : (h >= 31 ? 0u : ~((2u << h) - 1u));
    uint32_t prefix = kmin & pmask;
    for (int hi = h; hi >= 0; hi -= 8) {
      const int sh = hi >= 7 ? hi - 7 : 0;
      const uint32_t dmask = (2u << (hi - sh)) - 1u;
#pragma unroll
      for (int q = 0; q < 4; ++q) hist[4 * lane + q] = 0;
      wave_sync();
      for (uint32_t i0 = 0; i0 < M; i0 += 4 * 64) {
        uint32_t k[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t i = i0 + 64 * q + lane;
          k[q] = i < M ? tkey[start + i] : 0u;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t i = i0 + 64 * q + lane;
          if (i < M && ((k[q] ^ prefix) & pmask) == 0) atomicAdd(&hist[(k[q] >> sh) & dmask], 1u);
        }
      }
      wave_sync();
      // lane l holds digits 4l..4l+3: their counts, the lane total and the
      // exclusive prefix over lanes
      uint32_t c[4], tot = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = hist[4 * lane + q];
        tot += c[q];
      }
      uint32_t inc = tot;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
      }
      uint32_t exc = inc - tot, dsel = 0, bsel = 0;
      bool hit = false;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!hit && exc <= m && m < exc + c[q]) {
          hit = true;
          dsel = 4 * lane + q;
          bsel = exc;
        }
        exc += c[q];
      }
      const uint64_t hb = __ballot(hit);  // exactly one lane holds rank m
      const int src = __ffsll((long long)hb) - 1;
      const uint32_t d = __shfl(dsel, src), below = __shfl(bsel, src);
      m -= below;
      less += below;
      prefix |= d << sh;
      pmask |= dmask << sh;
      wave_sync();
    }
    key = prefix;  // all keys equal (h < 0): the common key, nothing below it
    split = less > 0;
  }
  if (lane == 0) {
    sflag[j] = split ? 1u : 0u;
    sel[3 * (size_t)j] = axis;
    sel[3 * (size_t)j + 1] = key;
    sel[3 * (size_t)j + 2] = less;
  }
}

// After the scan of the split flags: the list of splitting nodes, and the
// leaf record of every other node (slot leaf_base + number of non-splitting
// nodes before it).
__global__ __launch_bounds__(256) void kd_lists_kernel(Level lv, uint32_t active, const uint32_t *__restrict__ sflag,
                                                       const uint32_t *__restrict__ srank,
                                                       uint32_t *__restrict__ split_list,
                                                       uint32_t *__restrict__ leaf_start,
                                                       uint32_t *__restrict__ leaf_node, uint32_t leaf_base) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= active) return;
  if (sflag[j]) {
    split_list[srank[j]] = j;
  } else {
    const uint32_t slot = leaf_base + (j - srank[j]);
    leaf_start[slot] = lv.start[j];
    leaf_node[slot] = lv.id[j];
  }
}

// Partition of the splitting nodes, one workgroup per node of split_list:
// the segment is partitioned stably into tmp and copied back in place; the
// node's record and its two children are written.
__global__ __launch_bounds__(KD_THREADS) void kd_partition_kernel(
    uint32_t *__restrict__ perm, uint32_t *__restrict__ tmp, const uint32_t *__restrict__ tkey, Level lv, Level nx,
    const uint32_t *__restrict__ split_list, const uint32_t *__restrict__ srank, const uint32_t *__restrict__ sel,
    uint32_t node_base_next, npg_kd_node *__restrict__ nodes) {
  __shared__ uint32_t wl[KD_THREADS / 64], wr[KD_THREADS / 64];
  const uint32_t j = split_list[blockIdx.x];
  const uint32_t start = lv.start[j], M = lv.count[j], id = lv.id[j];
  const uint32_t axis = sel[3 * (size_t)j], key = sel[3 * (size_t)j + 1], less = sel[3 * (size_t)j + 2];
  const uint32_t c0 = node_base_next + 2 * srank[j];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t lbase = 0, rbase = 0;
  for (uint32_t r0 = 0; r0 < M; r0 += KD_THREADS) {
    const uint32_t i = r0 + threadIdx.x;
    const bool act = i < M;
    const bool left = act && tkey[start + i] < key;
    const uint64_t bl = __ballot(left), br = __ballot(act && !left);
    if (lane == 0) {
      wl[wave] = (uint32_t)__popcll(bl);
      wr[wave] = (uint32_t)__popcll(br);
    }
    __syncthreads();
    uint32_t ol = lbase, orr = rbase, tl = 0, tr = 0;
#pragma unroll
    for (int w = 0; w < KD_THREADS / 64; ++w) {
      if (w < wave) {
        ol += wl[w];
        orr += wr[w];
      }
      tl += wl[w];
      tr += wr[w];
    }
    if (act) {
      const uint32_t dst = left ? start + ol + (uint32_t)__popcll(bl & below)
                                : start + less + orr + (uint32_t)__popcll(br & below);
      tmp[dst] = perm[start + i];
    }
    lbase += tl;
    rbase += tr;
    __syncthreads();
  }
  // every read of the segment is done (barrier above): copy back in place
  for (uint32_t i = threadIdx.x; i < M; i += KD_THREADS) perm[start + i] = tmp[start + i];
  if (threadIdx.x == 0) {
    const float s = okey_inv(key);
    nodes[id].split = s;
    nodes[id].info = (c0 << 2) | axis;
    const uint32_t q0 = 2 * srank[j];
    nx.start[q0] = start;
    nx.count[q0] = less;
    nx.id[q0] = c0;
    nx.start[q0 + 1] = start + less;
    nx.count[q0 + 1] = M - less;
    nx.id[q0 + 1] = c0 + 1;
    const double *b = lv.box + 6 * (size_t)j;
    double *bl0 = nx.box + 6 * (size_t)q0, *br0 = nx.box + 6 * (size_t)(q0 + 1);
    for (int k = 0; k < 6; ++k) {
      bl0[k] = b[k];
      br0[k] = b[k];
    }
    bl0[3 + axis] = (double)s;
    br0[axis] = (double)s;
  }
}

__global__ __launch_bounds__(256) void kd_leaves_kernel(const uint32_t *__restrict__ start_sorted,
                                                        const uint32_t *__restrict__ node_sorted, uint32_t L,
                                                        const uint32_t *nvalid, uint32_t *__restrict__ leaf_off,
                                                        npg_kd_node *__restrict__ nodes) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < L) {
    leaf_off[k] = start_sorted[k];
    nodes[node_sorted[k]].split = 0.0f;
    nodes[node_sorted[k]].info = (k << 2) | 3u;
  }
  if (k == 0) leaf_off[L] = *nvalid;
}

__global__ __launch_bounds__(256) void kd_locate_kernel(GridDev g, const int32_t *__restrict__ root,
                                                        const npg_kd_node *__restrict__ nodes, uint32_t n_nodes,
                                                        const float *__restrict__ q, uint64_t n,
                                                        uint32_t *__restrict__ out, uint32_t *err) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const float p[3] = {q[3 * i], q[3 * i + 1], q[3 * i + 2]};
    uint32_t res = KD_NONE;
    if (!finite3(p[0], p[1], p[2])) {
      raise_err(err, ERR_RANGE);
    } else {
      const int32_t r = root[vox_id(g, p[0], p[1], p[2])];
      if (r >= 0) {
        uint32_t node = (uint32_t)r;
        for (int step = 0; step < 64; ++step) {  // depth <= 16: ends long before
          if (node >= n_nodes) {
            raise_err(err, ERR_RANGE);
            break;
          }
          const npg_kd_node nd = nodes[node];
          const uint32_t a = nd.info & 3u;
          if (a == 3u) {
            res = nd.info >> 2;
            break;
          }
          const float x = p[a] == 0.0f ? 0.0f : p[a];
          node = (nd.info >> 2) + (x < nd.split ? 0u : 1u);
        }
      }
    }
    out[i] = res;
  }
}

unsigned grid_for(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return (unsigned)(b ? (b < 65536 ? b : 65536) : 1);
}

int grid_params(npg_ctx *ctx, const npg_kdgrid_params *p, GridDev *g) {
  if (!p) return npg_fail(ctx, NPG_E_ARG, "kdgrid: null params");
  if (p->res < 1 || p->res > 1024) return npg_fail(ctx, NPG_E_ARG, "kdgrid: res %d outside [1,1024]", p->res);
  g->res = p->res;
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(p->lo[a]) || !std::isfinite(p->hi[a]) || !(p->hi[a] > p->lo[a]))
      return npg_fail(ctx, NPG_E_ARG, "kdgrid: box axis %d is empty or not finite", a);
    const double ext = (double)p->hi[a] - (double)p->lo[a];
    g->lo[a] = p->lo[a];
    g->invr[a] = (double)p->res / ext;
    g->step[a] = ext / (double)p->res;
  }
  return NPG_OK;
}

int take_err(npg_ctx *ctx, hipStream_t s, uint32_t *errw) {
  NPG_HIP_CHECK(ctx, hipMemcpyAsync(errw, ctx->err_dev, 4, hipMemcpyDeviceToHost, s));
  NPG_HIP_CHECK(ctx, hipStreamSynchronize(s));
  if (*errw) NPG_HIP_CHECK(ctx, hipMemsetAsync(ctx->err_dev, 0, 4, s));
  return NPG_OK;
}

}  // namespace

extern "C" int npg_mark_valid(npg_ctx *ctx, const npg_kdgrid_params *params, const float *pts_dev, uint64_t n,
                              uint8_t *valid_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  GridDev g;
  int rc = grid_params(ctx, params, &g);
  if (rc) return rc;
  if (!valid_dev || (n && !pts_dev)) return npg_fail(ctx, NPG_E_ARG, "mark_valid: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t nv = (uint64_t)g.res * g.res * g.res;
  NPG_HIP_CHECK(ctx, hipMemsetAsync(valid_dev, 0, nv, s));
  if (n) hipLaunchKernelGGL(kd_mark_kernel, dim3(grid_for(n)), dim3(256), 0, s, g, pts_dev, n, valid_dev, ctx->err_dev);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  return NPG_OK;
}

extern "C" int npg_build_kdgrid(npg_ctx *ctx, const npg_kdgrid_params *params, const float *pos_dev,
                                const float *normal_dev, uint64_t n, const uint8_t *valid_dev, uint32_t *perm_dev,
                                uint32_t *leaf_off_dev, int32_t *cell_root_dev, npg_kd_node *nodes_dev,
                                uint32_t max_leaves, uint32_t *n_leaves_out, uint32_t *n_nodes_out, void *stream) {
  if (!ctx) return NPG_E_ARG;
  GridDev g;
  int rc = grid_params(ctx, params, &g);
  if (rc) return rc;
  if (!n_leaves_out || !n_nodes_out) return npg_fail(ctx, NPG_E_ARG, "build_kdgrid: null count output");
  *n_leaves_out = 0;
  *n_nodes_out = 0;
  if (params->max_depth < 0 || params->max_depth > 16)
    return npg_fail(ctx, NPG_E_ARG, "build_kdgrid: max_depth %d outside [0,16]", params->max_depth);
  if (n > 0xffffffffull) return npg_fail(ctx, NPG_E_ARG, "build_kdgrid: n > 2^32-1");
  if (max_leaves == 0 || max_leaves >= (1u << 29))
    return npg_fail(ctx, NPG_E_ARG, "build_kdgrid: max_leaves %u outside [1, 2^29)", max_leaves);
  if (!leaf_off_dev || !cell_root_dev || !nodes_dev || (n && (!pos_dev || !perm_dev)))
    return npg_fail(ctx, NPG_E_ARG, "build_kdgrid: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t nvox = (uint64_t)g.res * g.res * g.res;
  const uint32_t sent = (uint32_t)nvox;
  const uint64_t m = n ? n : 1;
  const uint64_t cap = max_leaves;
  // scratch
  const size_t sort_work = npg_radix_work_bytes(std::max<uint64_t>(m, cap));
  size_t bytes = 5 * npg_align(4 * m) + npg_align(4 * (m + 1)) + sort_work;
  bytes += npg_align(4 * npg_scan_tmp_words(std::max<uint64_t>(m, cap)));
  bytes += 2 * (3 * npg_align(4 * cap) + npg_align(48 * cap));   // two levels
  bytes += 2 * npg_align(4 * (cap + 1)) + npg_align(12 * cap) + npg_align(4 * cap);  // sflag, srank, sel, lists
  bytes += 4 * npg_align(4 * cap) + npg_align(16);               // leaves, sorted leaves, counters
  void *scr = nullptr;
  rc = npg_scratch(ctx, bytes, s, &scr);
  if (rc) return rc;
  Carver cv(scr);
  uint32_t *key = cv.take<uint32_t>(m), *ks = cv.take<uint32_t>(m);
  uint32_t *pa = cv.take<uint32_t>(m);  // partition staging
  uint32_t *tkey = cv.take<uint32_t>(m), *flag = cv.take<uint32_t>(m);
  uint32_t *seg = cv.take<uint32_t>(m + 1);
  void *work = cv.take<char>(sort_work);
  uint32_t *stmp = cv.take<uint32_t>(npg_scan_tmp_words(std::max<uint64_t>(m, cap)));
  Level lv[2];
  for (auto &l : lv) {
    l.start = cv.take<uint32_t>(cap);
    l.count = cv.take<uint32_t>(cap);
    l.id = cv.take<uint32_t>(cap);
    l.box = cv.take<double>(6 * cap);
  }
  uint32_t *sflag = cv.take<uint32_t>(cap + 1), *srank = cv.take<uint32_t>(cap + 1);
  uint32_t *sel = cv.take<uint32_t>(3 * cap);
  uint32_t *big = cv.take<uint32_t>(cap);  // big-node list, then the split list
  uint32_t *lstart = cv.take<uint32_t>(cap), *lnode = cv.take<uint32_t>(cap);
  uint32_t *lstart_s = cv.take<uint32_t>(cap), *lnode_s = cv.take<uint32_t>(cap);
  uint32_t *ctr = cv.take<uint32_t>(4);  // [0] photons in valid voxels, [1] big nodes of a level

  NPG_HIP_CHECK(ctx, hipMemsetAsync(ctr, 0, 16, s));
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(nvox)), dim3(256), 0, s, cell_root_dev, nvox, -1);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  uint32_t n0 = 0;
  if (n) {
    hipLaunchKernelGGL(kd_keys_kernel, dim3(grid_for(n)), dim3(256), 0, s, g, pos_dev, normal_dev, n, valid_dev,
                       sent, key, ctx->err_dev);
    NPG_HIP_CHECK(ctx, hipGetLastError());
    int bits = 1;
    while (bits < 32 && (1ull << bits) <= (uint64_t)sent) ++bits;
    NPG_HIP_CHECK(ctx, npg_radix_sort(key, nullptr, n, bits, ks, perm_dev, work, s));
    hipLaunchKernelGGL(kd_seg_kernel, dim3(grid_for(n)), dim3(256), 0, s, ks, n, sent, flag, ctr);
    NPG_HIP_CHECK(ctx, hipGetLastError());
    NPG_HIP_CHECK(ctx, npg_scan_u32(flag, n, seg, stmp, s));
    NPG_HIP_CHECK(ctx, hipMemcpyAsync(&n0, seg + n, 4, hipMemcpyDeviceToHost, s));
    uint32_t errw = 0;
    rc = take_err(ctx, s, &errw);  // synchronises: n0 is now valid
    if (rc) return rc;
    if (errw & ERR_RANGE) return npg_fail(ctx, NPG_E_RANGE, "build_kdgrid: a position or normal is not finite");
    if (n0 > max_leaves)
      return npg_fail(ctx, NPG_E_CAPACITY, "build_kdgrid: %u voxel roots exceed max_leaves %u", n0, max_leaves);
    if (n0) {
      hipLaunchKernelGGL(kd_roots_kernel, dim3(grid_for(n)), dim3(256), 0, s, g, ks, flag, seg, n, lv[0],
                         cell_root_dev);
      hipLaunchKernelGGL(kd_root_counts_kernel, dim3((n0 + 255) / 256), dim3(256), 0, s, lv[0], n0, ctr);
      NPG_HIP_CHECK(ctx, hipGetLastError());
    }
  }
  // levels
  uint32_t active = n0, nodes_total = n0;
  uint64_t emitted = 0;
  for (int depth = 0; active > 0; ++depth) {
    Level &cur = lv[depth & 1], &nxt = lv[(depth + 1) & 1];
    NPG_HIP_CHECK(ctx, hipMemsetAsync(ctr + 1, 0, 4, s));
    hipLaunchKernelGGL(kd_select_wave_kernel, dim3((active + 3) / 4), dim3(KD_THREADS), 0, s, pos_dev, normal_dev,
                       perm_dev, cur, active, depth, params->max_depth, params->split_count, params->split_var, tkey,
                       sflag, sel, big, ctr + 1, ctx->err_dev);
    hipLaunchKernelGGL(kd_select_kernel, dim3(std::min<uint32_t>(active, 2048)), dim3(KD_THREADS), 0, s, pos_dev,
                       normal_dev, perm_dev, cur, big, ctr + 1, depth, params->max_depth, params->split_count,
                       params->split_var, tkey, sflag, sel, ctx->err_dev);
    NPG_HIP_CHECK(ctx, hipGetLastError());
    NPG_HIP_CHECK(ctx, npg_scan_u32(sflag, active, srank, stmp, s));
    uint32_t nsplit = 0;
    NPG_HIP_CHECK(ctx, hipMemcpyAsync(&nsplit, srank + active, 4, hipMemcpyDeviceToHost, s));
    NPG_HIP_CHECK(ctx, hipStreamSynchronize(s));
    // leaves so far + this level's + at least one per child: the bound keeps
    // the next level's records and every leaf slot within max_leaves
    const uint32_t leaf_base = (uint32_t)emitted;
    emitted += active - nsplit;
    if (emitted + 2ull * nsplit > cap)
      return npg_fail(ctx, NPG_E_CAPACITY, "build_kdgrid: more than max_leaves %u leaves", max_leaves);
    hipLaunchKernelGGL(kd_lists_kernel, dim3((active + 255) / 256), dim3(256), 0, s, cur, active, sflag, srank, big,
                       lstart, lnode, leaf_base);
    if (nsplit)
      hipLaunchKernelGGL(kd_partition_kernel, dim3(nsplit), dim3(KD_THREADS), 0, s, perm_dev, pa, tkey, cur, nxt, big,
                         srank, sel, nodes_total, nodes_dev);
    NPG_HIP_CHECK(ctx, hipGetLastError());
    nodes_total += 2 * nsplit;
    active = 2 * nsplit;
  }
  uint32_t hc[2] = {0, 0}, errw = 0;
  NPG_HIP_CHECK(ctx, hipMemcpyAsync(hc, ctr, 8, hipMemcpyDeviceToHost, s));
  rc = take_err(ctx, s, &errw);
  if (rc) return rc;
  // the key pass has checked every position and every normal it needed
  if (errw & ERR_RANGE) return npg_fail(ctx, NPG_E_RANGE, "build_kdgrid: a normal is not finite");
  const uint32_t L = (uint32_t)emitted;
  if (L > max_leaves)
    return npg_fail(ctx, NPG_E_CAPACITY, "build_kdgrid: %u leaves exceed max_leaves %u", L, max_leaves);
  if (L) {
    int bits = 1;
    while (bits < 32 && (1ull << bits) <= (uint64_t)hc[0]) ++bits;
    NPG_HIP_CHECK(ctx, npg_radix_sort(lstart, lnode, L, bits, lstart_s, lnode_s, work, s));
  }
  hipLaunchKernelGGL(kd_leaves_kernel, dim3(L ? (L + 255) / 256 : 1), dim3(256), 0, s, lstart_s, lnode_s, L, ctr,
                     leaf_off_dev, nodes_dev);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  NPG_HIP_CHECK(ctx, hipStreamSynchronize(s));
  *n_leaves_out = L;
  *n_nodes_out = nodes_total;
  return NPG_OK;
}

extern "C" int npg_locate(npg_ctx *ctx, const npg_kdgrid_params *params, const int32_t *cell_root_dev,
                          const npg_kd_node *nodes_dev, uint32_t n_nodes, const float *q_dev, uint64_t n,
                          uint32_t *leaf_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  GridDev g;
  int rc = grid_params(ctx, params, &g);
  if (rc) return rc;
  if (n == 0) return NPG_OK;
  if (!cell_root_dev || !q_dev || !leaf_dev || (n_nodes && !nodes_dev))
    return npg_fail(ctx, NPG_E_ARG, "locate: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(kd_locate_kernel, dim3(grid_for(n)), dim3(256), 0, s, g, cell_root_dev, nodes_dev, n_nodes,
                     q_dev, n, leaf_dev, ctx->err_dev);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  return NPG_OK;
}
