// Adaptive octree over the unit box: photon -> leaf assignment.
//
// A cell at depth d is a run of 8^(Dmax-d) consecutive cells of the finest
// level in Morton order, so every count the split rule needs is a difference
// of one exclusive prefix over the finest-level histogram:
//   1. cells:    q = floor(p * 2^21) per axis (exact for float32 in [0,1)),
//                finest cell = Morton interleave of q >> (21 - Dmax), and a
//                histogram of the finest cells;
//   2. scan:     exclusive prefix of the histogram (cell start offsets);
//   3. decide:   for every finest cell, walk down from the root while the
//                ancestor's count exceeds the threshold (and depth < Dmax);
//                the first unsplit ancestor is the leaf; a leaf starts at its
//                first finest cell and exists if its count is non-zero;
//   4. number:   exclusive prefix of the leaf-start flags = leaf ids in
//                Morton order; leaf CSR offsets are the cell start offsets;
//   5. permute:  stable LSD radix sort of (leaf id, photon index), 8-bit
//                digits; ranks inside a wavefront come from ballots over the
//                digit bits, so equal keys keep their input order.
#include "npg_internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr int RS_THREADS = 256;
constexpr int RS_WAVE_ITEMS = 1024;                 // items per wavefront per tile
constexpr int RS_TILE = RS_WAVE_ITEMS * (RS_THREADS / 64);

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 8 bits -> every third bit
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) r |= ((v >> b) & 1u) << (3 * b);
  return r;
}

// cnt == nullptr: the histogram is left to cell_hist_kernel
__global__ __launch_bounds__(256) void cells_kernel(const float *__restrict__ pos, uint64_t n, int dmax,
                                                    uint32_t *__restrict__ cell, uint32_t *__restrict__ cnt,
                                                    uint32_t *err) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const float x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const bool ok = x >= 0.0f && x < 1.0f && y >= 0.0f && y < 1.0f && z >= 0.0f && z < 1.0f;
    uint32_t c = 0;
    if (ok) {
      const int sh = 21 - dmax;
      const uint32_t qx = (uint32_t)(x * 2097152.0f) >> sh;
      const uint32_t qy = (uint32_t)(y * 2097152.0f) >> sh;
      const uint32_t qz = (uint32_t)(z * 2097152.0f) >> sh;
      c = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
    } else {
      raise_err(err, ERR_RANGE);
    }
    cell[i] = c;
    if (cnt) atomicAdd(&cnt[c], 1u);
  }
}

// Finest-cell histogram without hot-spot atomics.  Photons of a clustered
// scene pile into few cells, and one global atomic per photon serialises on
// those addresses.  Workgroup (r, p) instead counts, in LDS, the cells of
// range r (HIST_RANGE consecutive cell ids) among the photons of slice p,
// then adds its non-zero counts to the global histogram: one global atomic
// per (workgroup, occupied cell).
constexpr int HIST_RANGE = 32768;  // cells per workgroup (128 KiB of LDS counters)
constexpr int HIST_THREADS = 1024;

__global__ __launch_bounds__(HIST_THREADS) void cell_hist_kernel(const uint32_t *__restrict__ cell, uint64_t n,
                                                                 uint32_t ncell, uint64_t per_slice,
                                                                 uint32_t *__restrict__ cnt) {
  extern __shared__ uint32_t h[];
  const uint32_t r0 = blockIdx.x * (uint32_t)HIST_RANGE;
  const uint32_t nr = min((uint32_t)HIST_RANGE, ncell - r0);
  for (uint32_t k = threadIdx.x; k < nr; k += HIST_THREADS) h[k] = 0u;
  __syncthreads();
  // per_slice is a multiple of 4, so every slice starts 16-byte aligned
  const uint64_t b = (uint64_t)blockIdx.y * per_slice;
  const uint64_t e = min(n, b + per_slice);
  const uint64_t e4 = b + ((e - b) & ~(uint64_t)3);
  const uint4 *c4 = reinterpret_cast<const uint4 *>(cell + b);
  for (uint64_t i = threadIdx.x; b + 4 * i < e4; i += HIST_THREADS) {
    const uint4 v = c4[i];
    const uint32_t c[4] = {v.x - r0, v.y - r0, v.z - r0, v.w - r0};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (c[j] < nr) atomicAdd(&h[c[j]], 1u);
  }
  for (uint64_t i = e4 + threadIdx.x; i < e; i += HIST_THREADS) {
    const uint32_t c = cell[i] - r0;
    if (c < nr) atomicAdd(&h[c], 1u);
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nr; k += HIST_THREADS)
    if (h[k]) atomicAdd(&cnt[r0 + k], h[k]);
}

// ---------------------------------------------------------------- scan
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// exclusive scan of one value per thread across a 256-thread block;
// returns the prefix and sets *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t ws[SCAN_THREADS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan_u32(v, lane);
  if (lane == 63) ws[wave] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < SCAN_THREADS / 64; ++w) {
    if (w < wave) before += ws[w];
    tot += ws[w];
  }
  __syncthreads();
  *total = tot;
  return before + incl - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void scan_reduce_kernel(const uint32_t *__restrict__ in, uint64_t n,
                                                                   uint32_t *__restrict__ bsum) {
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
  uint32_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const uint64_t i = base + (uint64_t)k * SCAN_THREADS + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// single-block exclusive scan of m block sums, in place
__global__ __launch_bounds__(SCAN_THREADS) void scan_sums_kernel(uint32_t *__restrict__ bsum, uint32_t m) {
  const uint32_t per = (m + SCAN_THREADS - 1) / SCAN_THREADS;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (uint32_t k = 0; k < per; ++k)
    if (b0 + k < m) s += bsum[b0 + k];
  uint32_t tot;
  uint32_t run = block_excl_scan(s, &tot);
  for (uint32_t k = 0; k < per; ++k)
    if (b0 + k < m) {
      const uint32_t v = bsum[b0 + k];
      bsum[b0 + k] = run;
      run += v;
    }
}

// out[i] = offset of the block + exclusive prefix inside the block; out[n] = total
__global__ __launch_bounds__(SCAN_THREADS) void scan_down_kernel(const uint32_t *__restrict__ in, uint64_t n,
                                                                 const uint32_t *__restrict__ bsum,
                                                                 uint32_t *__restrict__ out) {
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const uint64_t i = base + k;
    v[k] = i < n ? in[i] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t run = bsum[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const uint64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = bsum[blockIdx.x] + tot;
}

// ---------------------------------------------------------------- tree
__global__ void decide_kernel(const uint32_t *__restrict__ cstart, uint32_t ncell, int dmax, uint32_t T,
                              uint32_t *__restrict__ flag, uint8_t *__restrict__ ldepth) {
  for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < ncell; f += gridDim.x * blockDim.x) {
    int d = 0;
    uint32_t count = 0, span = 1;
    for (d = 0; d <= dmax; ++d) {
      const int sh = 3 * (dmax - d);
      span = 1u << sh;
      const uint32_t a = f >> sh;
      count = cstart[(a + 1) * span] - cstart[a * span];
      if (count <= T || d == dmax) break;
    }
    flag[f] = ((f & (span - 1)) == 0 && count > 0) ? 1u : 0u;
    ldepth[f] = (uint8_t)d;
  }
}

__global__ void emit_kernel(const uint32_t *__restrict__ cstart, const uint32_t *__restrict__ flag,
                            const uint32_t *__restrict__ lid, const uint8_t *__restrict__ ldepth, uint32_t ncell,
                            int dmax, uint32_t max_leaves, uint64_t n, uint32_t *__restrict__ leaf_off,
                            uint64_t *__restrict__ key, uint8_t *__restrict__ depth) {
  for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < ncell; f += gridDim.x * blockDim.x) {
    if (!flag[f]) continue;
    const uint32_t id = lid[f];
    if (id >= max_leaves) continue;
    leaf_off[id] = cstart[f];
    if (key) key[id] = (uint64_t)f << (63 - 3 * dmax);
    if (depth) depth[id] = ldepth[f];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t L = lid[ncell];
    if (L <= max_leaves) leaf_off[L] = (uint32_t)n;
  }
}

// leaf id of every finest cell: the number of leaf starts up to and
// including it, minus one
__global__ void cell_leaf_kernel(const uint32_t *__restrict__ lid, const uint32_t *__restrict__ flag,
                                 uint32_t ncell, uint32_t *__restrict__ leafc) {
  for (uint32_t f = blockIdx.x * blockDim.x + threadIdx.x; f < ncell; f += gridDim.x * blockDim.x)
    leafc[f] = lid[f] + flag[f] - 1u;
}

// leaf_of[i] = leafc[cell[i]], four photons per thread and step (cell is
// scratch, 256-byte aligned; leaf_of takes 16-byte stores when aligned)
__global__ void leaf_of_kernel(const uint32_t *__restrict__ cell, uint64_t n, const uint32_t *__restrict__ leafc,
                               uint32_t *__restrict__ leaf_of, int vec_store) {
  const uint64_t n4 = n / 4;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n4;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint4 c = reinterpret_cast<const uint4 *>(cell)[i];
    const uint4 v = make_uint4(leafc[c.x], leafc[c.y], leafc[c.z], leafc[c.w]);
    if (vec_store) {
      reinterpret_cast<uint4 *>(leaf_of)[i] = v;
    } else {
      leaf_of[4 * i] = v.x;
      leaf_of[4 * i + 1] = v.y;
      leaf_of[4 * i + 2] = v.z;
      leaf_of[4 * i + 3] = v.w;
    }
  }
  const uint64_t t = 4 * n4 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t < n) leaf_of[t] = leafc[cell[t]];
}

// ---------------------------------------------------------- radix sort
__global__ __launch_bounds__(RS_THREADS) void rs_hist_kernel(const uint32_t *__restrict__ key, uint64_t n, int shift,
                                                             uint32_t nblocks, uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * RS_TILE;
  for (int k = threadIdx.x; k < RS_TILE; k += RS_THREADS) {
    const uint64_t i = base + k;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Between two passes the payload is one 16-byte record per photon
// (direction, weight); the first pass reads the caller's arrays, the last
// writes them.  Each item then costs one or two wide accesses per pass
// instead of four single words (a load whose 64 lanes hit 64 different
// lines costs the same at any width).
struct Payload {
  const float *dir_in = nullptr;
  const uint32_t *w_in = nullptr;
  const uint4 *rec_in = nullptr;
  float *dir_out = nullptr;
  uint32_t *w_out = nullptr;
  uint4 *rec_out = nullptr;
  __device__ bool on() const { return dir_in || rec_in; }
};
struct Dir3 {
  float x, y, z;
};

// Stable scatter of one 4096-item tile of an LSD radix pass (the tile of
// rs_hist_kernel).  Each item's key, value (the item index when vals is
// NULL) and payload are read in item order (coalesced), ordered by digit in
// LDS (ranks from wavefront ballots; waves and rounds in item order, so equal
// digits keep their input order), then streamed out: consecutive LDS
// entries of one digit go to consecutive global positions, so the writes
// form runs instead of single words.  1024 threads (16 wavefronts of 256
// items each); each wavefront issues the loads of its four rounds before
// ranking the first.  key_out == NULL: the keys are not written (the last
// pass).  PL: the payload (a photon's direction and weight, moved with the
// permutation) is moved too.
constexpr int RSP_THREADS = 1024;
constexpr int RSP_WAVES = RSP_THREADS / 64;
constexpr int RSP_WAVE_ITEMS = RS_TILE / RSP_WAVES;  // 256
constexpr int RSP_ROUNDS = RSP_WAVE_ITEMS / 64;      // 4

template <bool PL>
__global__ __launch_bounds__(RSP_THREADS) void rs_scatter_pl_kernel(const uint32_t *__restrict__ key,
                                                                   const uint32_t *__restrict__ vals, uint64_t n,
                                                                   int shift, uint32_t nblocks,
                                                                   const uint32_t *__restrict__ offs,
                                                                   uint32_t *__restrict__ key_out,
                                                                   uint32_t *__restrict__ val_out, Payload pl) {
  __shared__ uint32_t cnt[RSP_WAVES][256];
  __shared__ uint32_t tile_off[256], gdst[256], ws[4];
  __shared__ uint32_t lkey[RS_TILE], lval[RS_TILE];
  __shared__ uint4 lrec[PL ? RS_TILE : 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < RSP_WAVES * 256; k += RSP_THREADS) (&cnt[0][0])[k] = 0;
  const uint64_t tbase = (uint64_t)blockIdx.x * RS_TILE;
  const uint64_t wbase = tbase + (uint64_t)wave * RSP_WAVE_ITEMS;
  // this wavefront's items: keys, values and payload, loaded in order
  uint32_t kk[RSP_ROUNDS], vv[RSP_ROUNDS];
  uint4 rr[PL ? RSP_ROUNDS : 1];
#pragma unroll
  for (int r = 0; r < RSP_ROUNDS; ++r) {
    const uint64_t i = wbase + r * 64 + lane;
    const bool act = i < n;
    kk[r] = act ? key[i] : 0u;
    vv[r] = act ? (vals ? vals[i] : (uint32_t)i) : 0u;
    if constexpr (PL) {
      rr[r] = make_uint4(0, 0, 0, 0);
      if (act) {
        if (pl.rec_in) {
          rr[r] = pl.rec_in[i];
        } else {
          const Dir3 d = reinterpret_cast<const Dir3 *>(pl.dir_in)[i];
          rr[r] = make_uint4(__float_as_uint(d.x), __float_as_uint(d.y), __float_as_uint(d.z), pl.w_in[i]);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RSP_ROUNDS; ++r)
    if (wbase + r * 64 + lane < n) atomicAdd(&cnt[wave][(kk[r] >> shift) & 255u], 1u);
  __syncthreads();
  if (threadIdx.x < 256) {  // digit d: its tile count, exclusive scan, per-wave starts
    const int d = threadIdx.x;
    uint32_t c = 0;
    for (int w = 0; w < RSP_WAVES; ++w) c += cnt[w][d];
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (lane == 63) ws[wave] = incl;
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    const int d = threadIdx.x;
    uint32_t c = 0;
    for (int w = 0; w < RSP_WAVES; ++w) c += cnt[w][d];
    uint32_t run = 0;
    for (int w = 0; w < wave; ++w) run += ws[w];
    // incl - c recomputed from the wave's scan: the prefix within the wave
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    run += incl - c;
    tile_off[d] = run;
    gdst[d] = offs[(uint64_t)d * nblocks + blockIdx.x];
    for (int w = 0; w < RSP_WAVES; ++w) {
      const uint32_t cw = cnt[w][d];
      cnt[w][d] = run;
      run += cw;
    }
  }
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < RSP_ROUNDS; ++r) {
    const bool act = wbase + r * 64 + lane < n;
    const uint32_t dg = (kk[r] >> shift) & 255u;
    uint64_t mask = __ballot(act);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot(((dg >> b) & 1u) != 0);
      mask &= ((dg >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(mask & below);
    const uint32_t tot = (uint32_t)__popcll(mask);
    uint32_t basev = 0;
    if (act) basev = cnt[wave][dg];
    __builtin_amdgcn_wave_barrier();
    if (act) {
      const uint32_t pos = basev + rank;
      lkey[pos] = kk[r];
      lval[pos] = vv[r];
      if constexpr (PL) lrec[pos] = rr[r];
      if (rank == 0) cnt[wave][dg] = basev + tot;
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  const uint32_t nt = (uint32_t)min((uint64_t)RS_TILE, n - tbase);
  for (uint32_t j = threadIdx.x; j < nt; j += RSP_THREADS) {
    const uint32_t k2 = lkey[j];
    const uint32_t dg = (k2 >> shift) & 255u;
    const uint32_t pos = gdst[dg] + (j - tile_off[dg]);
    if (key_out) key_out[pos] = k2;
    val_out[pos] = lval[j];
    if constexpr (PL) {
      const uint4 q = lrec[j];
      if (pl.rec_out) {
        pl.rec_out[pos] = q;
      } else {
        reinterpret_cast<Dir3 *>(pl.dir_out)[pos] = Dir3{__uint_as_float(q.x), __uint_as_float(q.y), __uint_as_float(q.z)};
        pl.w_out[pos] = q.w;
      }
    }
  }
}

unsigned grid_of(uint64_t n, unsigned per = 256, unsigned cap = 65536) {
  const uint64_t b = (n + per - 1) / per;
  return (unsigned)(b < cap ? (b ? b : 1) : cap);
}

}  // namespace

// exclusive scan of n u32 into out[0..n] (out[n] = total); tmp holds
// ceil(n / SCAN_TILE) block sums
static hipError_t scan_u32(const uint32_t *in, uint64_t n, uint32_t *out, uint32_t *tmp, hipStream_t s) {
  const uint32_t nb = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE);
  const uint32_t nbx = nb ? nb : 1;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nbx), dim3(SCAN_THREADS), 0, s, in, n, tmp);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(SCAN_THREADS), 0, s, tmp, nbx);
  hipLaunchKernelGGL(scan_down_kernel, dim3(nbx), dim3(SCAN_THREADS), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

size_t npg_scan_tmp_words(uint64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t npg_scan_u32(const uint32_t *in, uint64_t n, uint32_t *out, uint32_t *tmp, hipStream_t s) {
  return scan_u32(in, n, out, tmp, s);
}

size_t npg_radix_work_bytes(uint64_t n) {
  const uint64_t nb = (n + RS_TILE - 1) / RS_TILE, nhist = 256 * (nb ? nb : 1);
  const uint64_t m = n ? n : 1;
  return 4 * npg_align(4 * m) + 2 * npg_align(4 * (nhist + 1)) + npg_align(4 * npg_scan_tmp_words(nhist));
}

hipError_t npg_radix_sort(const uint32_t *keys_in, const uint32_t *vals_in, uint64_t n, int bits,
                          uint32_t *keys_out, uint32_t *vals_out, void *work, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (bits < 1 || bits > 32) return hipErrorInvalidValue;
  const uint32_t nb = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
  const uint64_t nhist = 256ull * nb;
  Carver cv(work);
  uint32_t *ka = cv.take<uint32_t>(n), *kb = cv.take<uint32_t>(n);
  uint32_t *va = cv.take<uint32_t>(n), *vb = cv.take<uint32_t>(n);
  uint32_t *hist = cv.take<uint32_t>(nhist + 1), *offs = cv.take<uint32_t>(nhist + 1);
  uint32_t *btmp = cv.take<uint32_t>(npg_scan_tmp_words(nhist));
  const int passes = (bits + 7) / 8;
  const uint32_t *kin = keys_in, *vin = vals_in;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    uint32_t *kout = last ? keys_out : ((p & 1) ? kb : ka);
    uint32_t *vout = last ? vals_out : ((p & 1) ? vb : va);
    hipLaunchKernelGGL(rs_hist_kernel, dim3(nb), dim3(RS_THREADS), 0, s, kin, n, 8 * p, nb, hist);
    hipError_t e = scan_u32(hist, nhist, offs, btmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rs_scatter_pl_kernel<false>, dim3(nb), dim3(RSP_THREADS), 0, s, kin, vin, n, 8 * p, nb, offs,
                       kout, vout, Payload{});
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    kin = kout;
    vin = vout;
  }
  return hipSuccess;
}

// The octree build; pl.dir_out non-null: the photons' directions and
// weights are moved with the permutation into leaf order.
static int build_hierarchy(npg_ctx *ctx, const float *pos_dev, uint64_t n, const npg_hier_params *params,
                           uint32_t *perm_dev, uint32_t *leaf_of_dev, uint32_t *leaf_off_dev,
                           uint64_t *leaf_key_dev, uint8_t *leaf_depth_dev, uint32_t max_leaves,
                           uint32_t *n_leaves_out, void *stream, const Payload &pl) {
  if (!ctx) return NPG_E_ARG;
  if (!params || !n_leaves_out) return npg_fail(ctx, NPG_E_ARG, "build_hierarchy: null argument");
  if (params->max_depth < 0 || params->max_depth > 8)
    return npg_fail(ctx, NPG_E_ARG, "build_hierarchy: max_depth %d outside [0,8]", params->max_depth);
  if (n > 0xffffffffull) return npg_fail(ctx, NPG_E_ARG, "build_hierarchy: n > 2^32-1");
  if (max_leaves == 0) return npg_fail(ctx, NPG_E_ARG, "build_hierarchy: max_leaves = 0");
  if (!leaf_off_dev || (n && (!pos_dev || !perm_dev)))
    return npg_fail(ctx, NPG_E_ARG, "build_hierarchy: null pointer");
  int rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int D = params->max_depth;
  const uint32_t ncell = 1u << (3 * D);
  const uint32_t nb_rs = (uint32_t)((n + RS_TILE - 1) / RS_TILE);
  const uint64_t nhist = (uint64_t)256 * (nb_rs ? nb_rs : 1);
  const uint64_t scan_max = std::max<uint64_t>(std::max<uint64_t>(ncell + 1, nhist), 1);
  // scratch
  size_t bytes = 0;
  bytes += npg_align(4 * (n ? n : 1));             // cell
  bytes += npg_align(4 * ((uint64_t)ncell + 1));   // cnt
  bytes += npg_align(4 * ((uint64_t)ncell + 1));   // cstart
  bytes += npg_align(4 * ((uint64_t)ncell + 1));   // flag
  bytes += npg_align(4 * ((uint64_t)ncell + 1));   // lid
  bytes += npg_align((uint64_t)ncell + 1);         // ldepth
  bytes += npg_align(4 * (n ? n : 1)) * 3;         // leaf_of (own), keys A, keys B
  bytes += npg_align(4 * (n ? n : 1));             // vals tmp
  if (pl.dir_out) bytes += 2 * npg_align(16 * (n ? n : 1));  // payload records between the passes
  bytes += npg_align(4 * (nhist + 1)) * 2;         // hist, offs
  bytes += npg_align(4 * ((scan_max + SCAN_TILE - 1) / SCAN_TILE + 1));
  void *scr = nullptr;
  rc = npg_scratch(ctx, bytes, s, &scr);
  if (rc) return rc;
  Carver cv(scr);
  uint32_t *cell = cv.take<uint32_t>(n ? n : 1);
  uint32_t *cnt = cv.take<uint32_t>((uint64_t)ncell + 1);
  uint32_t *cstart = cv.take<uint32_t>((uint64_t)ncell + 1);
  uint32_t *flag = cv.take<uint32_t>((uint64_t)ncell + 1);
  uint32_t *lid = cv.take<uint32_t>((uint64_t)ncell + 1);
  uint8_t *ldepth = cv.take<uint8_t>((uint64_t)ncell + 1);
  uint32_t *lof_own = cv.take<uint32_t>(n ? n : 1);
  uint32_t *ka = cv.take<uint32_t>(n ? n : 1);
  uint32_t *kb = cv.take<uint32_t>(n ? n : 1);
  uint32_t *vt = cv.take<uint32_t>(n ? n : 1);
  uint4 *rec[2] = {pl.dir_out ? cv.take<uint4>(n ? n : 1) : nullptr, pl.dir_out ? cv.take<uint4>(n ? n : 1) : nullptr};
  uint32_t *hist = cv.take<uint32_t>(nhist + 1);
  uint32_t *offs = cv.take<uint32_t>(nhist + 1);
  uint32_t *btmp = cv.take<uint32_t>((scan_max + SCAN_TILE - 1) / SCAN_TILE + 1);

  NPG_HIP_CHECK(ctx, hipMemsetAsync(cnt, 0, 4 * ((size_t)ncell + 1), s));
  // up to 8 cell ranges (depth <= 6) the LDS histogram reads the cell ids
  // once per range; deeper trees spread their photons over enough cells for
  // direct atomics
  const uint32_t nranges = (ncell + HIST_RANGE - 1) / HIST_RANGE;
  const bool lds_hist = nranges <= 8;
  if (n)
    hipLaunchKernelGGL(cells_kernel, dim3(grid_of(n)), dim3(256), 0, s, pos_dev, n, D, cell,
                       lds_hist ? nullptr : cnt, ctx->err_dev);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  if (n && lds_hist) {
    static std::atomic<uint64_t> attr{0};
    if (npg_first_on_device(attr))
      NPG_HIP_CHECK(ctx, hipFuncSetAttribute((const void *)cell_hist_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, HIST_RANGE * 4));
    // about 1024 workgroups; slices of at least 16k photons, multiples of 4
    const uint64_t slices = std::max<uint64_t>(1, std::min<uint64_t>(1024 / nranges, (n + 16383) / 16384));
    const uint64_t per_slice = ((n + slices - 1) / slices + 3) & ~(uint64_t)3;
    const uint32_t ns = (uint32_t)((n + per_slice - 1) / per_slice);
    hipLaunchKernelGGL(cell_hist_kernel, dim3(nranges, ns), dim3(HIST_THREADS), HIST_RANGE * 4, s, cell, n, ncell,
                       per_slice, cnt);
    NPG_HIP_CHECK(ctx, hipGetLastError());
  }
  NPG_HIP_CHECK(ctx, scan_u32(cnt, ncell, cstart, btmp, s));
  hipLaunchKernelGGL(decide_kernel, dim3(grid_of(ncell)), dim3(256), 0, s, cstart, ncell, D, params->split_count,
                     flag, ldepth);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  NPG_HIP_CHECK(ctx, scan_u32(flag, ncell, lid, btmp, s));
  hipLaunchKernelGGL(emit_kernel, dim3(grid_of(ncell)), dim3(256), 0, s, cstart, flag, lid, ldepth, ncell, D,
                     max_leaves, n, leaf_off_dev, leaf_key_dev, leaf_depth_dev);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  uint32_t L = 0, errw = 0;
  NPG_HIP_CHECK(ctx, hipMemcpyAsync(&L, lid + ncell, 4, hipMemcpyDeviceToHost, s));
  NPG_HIP_CHECK(ctx, hipMemcpyAsync(&errw, ctx->err_dev, 4, hipMemcpyDeviceToHost, s));
  NPG_HIP_CHECK(ctx, hipStreamSynchronize(s));
  *n_leaves_out = L;
  if (errw & ERR_RANGE) {
    NPG_HIP_CHECK(ctx, hipMemsetAsync(ctx->err_dev, 0, 4, s));
    return npg_fail(ctx, NPG_E_RANGE, "build_hierarchy: a position is outside [0,1)^3 or not finite");
  }
  if (L > max_leaves)
    return npg_fail(ctx, NPG_E_CAPACITY, "build_hierarchy: %u leaves exceed max_leaves %u", L, max_leaves);
  if (n == 0) return NPG_OK;
  uint32_t *lof = leaf_of_dev ? leaf_of_dev : lof_own;
  uint32_t *leafc = cnt;  // the histogram is no longer needed
  hipLaunchKernelGGL(cell_leaf_kernel, dim3(grid_of(ncell)), dim3(256), 0, s, lid, flag, ncell, leafc);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  hipLaunchKernelGGL(leaf_of_kernel, dim3(grid_of((n + 3) / 4)), dim3(256), 0, s, cell, n, leafc, lof,
                     ((uintptr_t)lof & 15) == 0 ? 1 : 0);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  // stable radix sort of (leaf id, index) -> perm
  int bits = 1;
  while (bits < 32 && (1ull << bits) < L) ++bits;
  const int passes = (bits + 7) / 8;
  const uint32_t *kin = lof;
  const uint32_t *vin = nullptr;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    uint32_t *kout = last ? nullptr : ((p & 1) ? kb : ka);
    uint32_t *vout = last ? perm_dev : ((vin == vt) ? cell : vt);  // cell is free after leaf_of
    // payload: the caller's arrays into records, records into records
    // (alternating buffers), the last pass into the caller's outputs
    Payload step{};
    if (pl.dir_out) {
      if (p == 0) {
        step.dir_in = pl.dir_in;
        step.w_in = pl.w_in;
      } else {
        step.rec_in = rec[(p - 1) & 1];
      }
      if (last) {
        step.dir_out = pl.dir_out;
        step.w_out = pl.w_out;
      } else {
        step.rec_out = rec[p & 1];
      }
    }
    hipLaunchKernelGGL(rs_hist_kernel, dim3(nb_rs), dim3(RS_THREADS), 0, s, kin, n, 8 * p, nb_rs, hist);
    NPG_HIP_CHECK(ctx, scan_u32(hist, nhist, offs, btmp, s));
    if (pl.dir_out)
      hipLaunchKernelGGL(rs_scatter_pl_kernel<true>, dim3(nb_rs), dim3(RSP_THREADS), 0, s, kin, vin, n, 8 * p, nb_rs,
                         offs, kout, vout, step);
    else
      hipLaunchKernelGGL(rs_scatter_pl_kernel<false>, dim3(nb_rs), dim3(RSP_THREADS), 0, s, kin, vin, n, 8 * p,
                         nb_rs, offs, kout, vout, step);
    NPG_HIP_CHECK(ctx, hipGetLastError());
    kin = kout;
    vin = vout;
  }
  return NPG_OK;
}

extern "C" int npg_build_hierarchy(npg_ctx *ctx, const float *pos_dev, uint64_t n,
                                   const npg_hier_params *params, uint32_t *perm_dev,
                                   uint32_t *leaf_of_dev, uint32_t *leaf_off_dev,
                                   uint64_t *leaf_key_dev, uint8_t *leaf_depth_dev,
                                   uint32_t max_leaves, uint32_t *n_leaves_out, void *stream) {
  return build_hierarchy(ctx, pos_dev, n, params, perm_dev, leaf_of_dev, leaf_off_dev, leaf_key_dev,
                         leaf_depth_dev, max_leaves, n_leaves_out, stream, Payload{});
}

extern "C" int npg_build_hierarchy_sorted(npg_ctx *ctx, const float *pos_dev, const float *dir_dev,
                                          const uint32_t *w_dev, uint64_t n, const npg_hier_params *params,
                                          uint32_t *perm_dev, float *dir_sorted_dev, uint32_t *w_sorted_dev,
                                          uint32_t *leaf_off_dev, uint64_t *leaf_key_dev, uint8_t *leaf_depth_dev,
                                          uint32_t max_leaves, uint32_t *n_leaves_out, void *stream) {
  if (!ctx) return NPG_E_ARG;
  if (n && (!dir_dev || !w_dev || !dir_sorted_dev || !w_sorted_dev))
    return npg_fail(ctx, NPG_E_ARG, "build_hierarchy_sorted: null photon array");
  if (n && (dir_sorted_dev == dir_dev || w_sorted_dev == w_dev))
    return npg_fail(ctx, NPG_E_ARG, "build_hierarchy_sorted: the sorted photons cannot overwrite the input");
  Payload pl;
  pl.dir_in = dir_dev;
  pl.w_in = w_dev;
  pl.dir_out = dir_sorted_dev;
  pl.w_out = w_sorted_dev;
  return build_hierarchy(ctx, pos_dev, n, params, perm_dev, nullptr, leaf_off_dev, leaf_key_dev, leaf_depth_dev,
                         max_leaves, n_leaves_out, stream, pl);
}
