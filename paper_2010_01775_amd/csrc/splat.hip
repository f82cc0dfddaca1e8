// Photon binning into per-leaf energy/count maps, and the mean-1 input
// normalisation of the energy map.
//
// Splat: one workgroup per (leaf, band of rows).  The band's bins live in LDS
// as packed 64-bit words: bits 0..46 accumulate energy, bits 47..63 the
// photon count.  A photon adds (1 << 47) + w with one LDS atomic.  Packing is
// exact as long as a round covers at most 2^15 photons (energy < 2^47, count
// <= 2^15 < 2^17); after each round the words are drained into per-thread
// 64-bit registers, so leaves of any size are exact.  Integer sums make the
// result independent of the order photons are processed in.
#include "npg_internal.h"

namespace {

constexpr int SPLAT_THREADS = 1024;
constexpr int SPLAT_MAX_BINS = 16384;           // 128 KiB of packed words
constexpr uint32_t SPLAT_ROUND = 1u << 15;     // photons per drain round
constexpr int PACK_SHIFT = 47;
constexpr unsigned long long PACK_MASK = (1ull << PACK_SHIFT) - 1;

// Where a workgroup finds its leaf's photons: a CSR batch (one direction and
// weight array, offsets, optional permutation) or per-leaf descriptors
// (serving batches mix leaves of several requests).
struct CsrLeaves {
  const float *dir;
  const uint32_t *w;
  const uint32_t *perm;
  const uint32_t *off;
  __device__ void range(int leaf, uint32_t *b, uint32_t *e) const {
    *b = off[leaf];
    *e = off[leaf + 1];
  }
  __device__ uint32_t idx(int, uint32_t i) const { return perm ? perm[i] : i; }
  __device__ const float *dirs(int) const { return dir; }
  __device__ const uint32_t *ws(int) const { return w; }
};

struct DescLeaves {
  const npg_leaf_desc *d;
  __device__ void range(int leaf, uint32_t *b, uint32_t *e) const {
    *b = d[leaf].begin;
    *e = d[leaf].begin + d[leaf].count;
  }
  __device__ uint32_t idx(int, uint32_t i) const { return i; }
  __device__ const float *dirs(int leaf) const { return d[leaf].dir; }
  __device__ const uint32_t *ws(int leaf) const { return d[leaf].w; }
};

template <int BPT, int NT, class LS>
__global__ __launch_bounds__(NT) void splat_kernel(
    const float2 *__restrict__ bnd, LS src, int H, int W, int band_rows, uint64_t *__restrict__ energy,
    uint32_t *__restrict__ count, int accumulate, uint32_t *err) {
  extern __shared__ unsigned long long acc[];
  __shared__ float2 q4[256];
  const int leaf = blockIdx.x;
  const int row0 = blockIdx.y * band_rows;
  const int nb = band_rows * W;
  const int tid = threadIdx.x;
  for (int k = tid; k < nb; k += NT) acc[k] = 0ull;
  load_quarter(bnd, W, q4);
  unsigned long long e[BPT];
  uint32_t c[BPT];
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    e[j] = 0ull;
    c[j] = 0u;
  }
  uint32_t beg, end;
  src.range(leaf, &beg, &end);
  const float *dir = src.dirs(leaf);
  const uint32_t *w = src.ws(leaf);
  bool bad = false;
  __syncthreads();
  for (uint64_t r0 = beg; r0 < end; r0 += SPLAT_ROUND) {
    const uint32_t r1 = (uint32_t)min((uint64_t)end, r0 + SPLAT_ROUND);
    // PB photons per thread and step: all their loads are issued before
    // the first bin is computed
    constexpr int PB = 2;
    for (uint32_t i0 = (uint32_t)r0 + tid; i0 < r1; i0 += PB * NT) {
      float x[PB], y[PB], z[PB];
      uint32_t wp[PB];
#pragma unroll
      for (int j = 0; j < PB; ++j) {
        const uint32_t i = i0 + j * NT;
        const uint32_t p = src.idx(leaf, i < r1 ? i : i0);
        x[j] = dir[3 * (size_t)p];
        y[j] = dir[3 * (size_t)p + 1];
        z[j] = dir[3 * (size_t)p + 2];
        wp[j] = w[p];
      }
#pragma unroll
      for (int j = 0; j < PB; ++j) {
        if (i0 + j * NT >= r1) continue;
        if (!finite3(x[j], y[j], z[j])) {
          bad = true;
          continue;
        }
        const int iz = z_row(z[j], H) - row0;
        if (iz < 0 || iz >= band_rows) continue;
        const int k = iz * W + phi_sector(q4, x[j], y[j], W);
        atomicAdd(&acc[k], (1ull << PACK_SHIFT) + (unsigned long long)wp[j]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int k = tid + j * NT;
      if (k < nb) {
        const unsigned long long v = acc[k];
        acc[k] = 0ull;
        e[j] += v & PACK_MASK;
        c[j] += (uint32_t)(v >> PACK_SHIFT);
      }
    }
    __syncthreads();
  }
  if (bad && blockIdx.y == 0) raise_err(err, ERR_RANGE);
  const size_t base = ((size_t)leaf * H + row0) * W;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int k = tid + j * NT;
    if (k < nb) {
      if (accumulate) {
        energy[base + k] += e[j];
        if (count) count[base + k] += c[j];
      } else {
        energy[base + k] = e[j];
        if (count) count[base + k] = c[j];
      }
    }
  }
}

template <int BPT, int NT, class LS>
hipError_t launch_splat_t(const float2 *bnd, const LS &src, uint32_t L, int H, int W, int band_rows,
                          uint64_t *energy, uint32_t *count, int accumulate, uint32_t *err, hipStream_t s) {
  const size_t lds = sizeof(unsigned long long) * (size_t)band_rows * W;
  static std::atomic<uint64_t> attr{0};
  if (npg_first_on_device(attr)) {
    hipError_t e = hipFuncSetAttribute((const void *)splat_kernel<BPT, NT, LS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       SPLAT_MAX_BINS * sizeof(unsigned long long));
    if (e != hipSuccess) return e;
  }
  dim3 grid(L, H / band_rows);
  hipLaunchKernelGGL((splat_kernel<BPT, NT, LS>), grid, dim3(NT), lds, s, bnd, src, H, W, band_rows,
                     energy, count, accumulate, err);
  return hipGetLastError();
}

// Maps of up to 4096 bins take 512-thread workgroups (four fit a CU, so a
// 1024-leaf batch is resident at once); larger bands 1024 threads.
template <class LS>
hipError_t launch_splat_any(const float2 *bnd, const LS &src, uint32_t L, int H, int W, uint64_t *energy,
                            uint32_t *count, int accumulate, uint32_t *err, hipStream_t s) {
  int band_rows = H;
  while (band_rows * W > SPLAT_MAX_BINS) band_rows >>= 1;
  const int nb = band_rows * W;
  if (nb <= 4096) {
    switch ((nb + 511) / 512) {
      case 1: return launch_splat_t<1, 512>(bnd, src, L, H, W, band_rows, energy, count, accumulate, err, s);
      case 2: return launch_splat_t<2, 512>(bnd, src, L, H, W, band_rows, energy, count, accumulate, err, s);
      case 4: return launch_splat_t<4, 512>(bnd, src, L, H, W, band_rows, energy, count, accumulate, err, s);
      default: return launch_splat_t<8, 512>(bnd, src, L, H, W, band_rows, energy, count, accumulate, err, s);
    }
  }
  switch ((nb + SPLAT_THREADS - 1) / SPLAT_THREADS) {
    case 8: return launch_splat_t<8, SPLAT_THREADS>(bnd, src, L, H, W, band_rows, energy, count, accumulate, err, s);
    default: return launch_splat_t<16, SPLAT_THREADS>(bnd, src, L, H, W, band_rows, energy, count, accumulate, err, s);
  }
}

// Per-leaf energy total (exact u64 sum), stored as binary64.
__global__ __launch_bounds__(256) void leaf_total_kernel(const uint64_t *__restrict__ energy, int HW,
                                                         double *__restrict__ tot) {
  __shared__ unsigned long long part[4];
  const int leaf = blockIdx.x;
  const uint64_t *e = energy + (size_t)leaf * HW;
  unsigned long long s = 0;
  for (int k = threadIdx.x; k < HW; k += 256) s += e[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) tot[leaf] = (double)(part[0] + part[1] + part[2] + part[3]);
}

// x = H*W*E / total in binary64, rounded to float32; zero map for total 0.
__global__ void apply_scale_kernel(const uint64_t *__restrict__ energy, const double *__restrict__ tot,
                                   int HW, int log2HW, size_t n, float *__restrict__ x) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double t = tot[i >> log2HW];
    x[i] = t > 0.0 ? (float)((double)HW * (double)energy[i] / t) : 0.0f;
  }
}

}  // namespace

hipError_t launch_splat(const float2 *bnd, const float *dir, const uint32_t *w, const uint32_t *perm,
                        const uint32_t *off, uint32_t L, int H, int W, uint64_t *energy,
                        uint32_t *count, int accumulate, uint32_t *err, hipStream_t s) {
  return launch_splat_any(bnd, CsrLeaves{dir, w, perm, off}, L, H, W, energy, count, accumulate, err, s);
}

hipError_t launch_splat_desc(const float2 *bnd, const npg_leaf_desc *d, uint32_t L, int H, int W,
                             uint64_t *energy, uint32_t *err, hipStream_t s) {
  return launch_splat_any(bnd, DescLeaves{d}, L, H, W, energy, nullptr, 0, err, s);
}

hipError_t launch_leaf_scale(const uint64_t *energy, uint32_t L, int HW, double *tot, hipStream_t s) {
  hipLaunchKernelGGL(leaf_total_kernel, dim3(L), dim3(256), 0, s, energy, HW, tot);
  return hipGetLastError();
}

hipError_t launch_apply_scale(const uint64_t *energy, const double *tot, uint32_t L, int HW,
                              float *x, hipStream_t s) {
  const size_t n = (size_t)L * HW;
  int log2HW = 0;
  while ((1 << log2HW) < HW) ++log2HW;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(apply_scale_kernel, dim3(blocks), dim3(256), 0, s, energy, tot, HW, log2HW, n, x);
  return hipGetLastError();
}
