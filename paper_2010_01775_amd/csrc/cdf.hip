// pdf and marginal/conditional CDF tables of each leaf's density.
//
// One workgroup (4 wavefronts) per leaf.  Every sum and prefix is formed in
// binary64 and only the stored tables are rounded to float32:
//   S = sum s;  p = s / S;  pdf = p*H*W/(4 pi)
//   row mass m_i = sum_j p_ij, marginal M_i = sum_{i'<i} m_i' (M_H = 1)
//   conditional C_ij = sum_{j'<j} p_ij' / m_i (C_iW = 1; j/W if m_i = 0)
// The quotients are taken as products with binary64 reciprocals of S and
// m_i (one more binary64 rounding, far below the float32 rounding of the
// stored values).  A row is scanned by one wavefront in slices of 64
// consecutive bins (coalesced loads and stores): a wavefront scan per slice
// plus the running total of the slices before it.
#include <math.h>

#include "npg_internal.h"

namespace {

constexpr int CDF_THREADS = 256;
constexpr double FOUR_PI = 4.0 * M_PI;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// exclusive prefix over the 64 lanes
__device__ __forceinline__ double wave_excl_scan(double v, int lane) {
  double incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  return incl - v;
}

// Output tables of leaf l: contiguous batch arrays, or per-leaf pointers.
struct BatchOut {
  float *pdf, *marg, *cond;
  double *total;
  __device__ void get(int l, int H, int W, float **p, float **m, float **c, double **t) const {
    *p = pdf + (size_t)l * H * W;
    *m = marg + (size_t)l * (H + 1);
    *c = cond + (size_t)l * H * (W + 1);
    *t = total ? total + l : nullptr;
  }
};
struct DescOut {
  const npg_leaf_desc *d;
  __device__ void get(int l, int, int, float **p, float **m, float **c, double **t) const {
    *p = d[l].pdf;
    *m = d[l].marg;
    *c = d[l].cond;
    *t = d[l].total;
  }
};

template <class OUT, int SEG>
__global__ __launch_bounds__(CDF_THREADS) void cdf_kernel(const float *__restrict__ dens, int H, int W, OUT out,
                                                          uint32_t *err) {
  extern __shared__ double rowmass[];  // [H]
  __shared__ double red[4];
  __shared__ int bad_s;
  const int leaf = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t HW = (size_t)H * W;
  const float *s = dens + leaf * HW;
  if (tid == 0) bad_s = 0;
  __syncthreads();
  // total S
  double acc = 0.0;
  int bad = 0;
  for (size_t k = tid; k < HW; k += CDF_THREADS) {
    const float v = s[k];
    if (!(v >= 0.0f) || !isfinite(v)) bad = 1;
    acc += (double)v;
  }
  acc = wave_sum(acc);
  if (lane == 0) red[wave] = acc;
  if (bad) atomicOr(&bad_s, 1);
  __syncthreads();
  const double S = red[0] + red[1] + red[2] + red[3];
  float *pl, *ml, *cl;
  double *tl;
  out.get(leaf, H, W, &pl, &ml, &cl, &tl);
  if (bad_s || !(S > 0.0) || !isfinite(S)) {
    const float qnan = __int_as_float(0x7fc00000);
    for (size_t k = tid; k < HW; k += CDF_THREADS) pl[k] = qnan;
    for (int k = tid; k <= H; k += CDF_THREADS) ml[k] = qnan;
    for (size_t k = tid; k < (size_t)H * (W + 1); k += CDF_THREADS) cl[k] = qnan;
    if (tid == 0) {
      if (tl) *tl = 0.0;
      raise_err(err, ERR_RANGE);
    }
    return;
  }
  const double invS = 1.0 / S;
  const double pdf_k = (double)HW / FOUR_PI;
  // rows: one wavefront per row, bins j = 64 t + lane of slice t
  for (int i = wave; i < H; i += 4) {
    const float *srow = s + (size_t)i * W;
    float *prow = pl + (size_t)i * W;
    double c[SEG];  // exclusive prefix of p over the row at this lane's bins
    double run = 0.0;
#pragma unroll
    for (int t = 0; t < SEG; ++t) {
      const int j = 64 * t + lane;
      const double p = j < W ? (double)srow[j] * invS : 0.0;
      if (j < W) prow[j] = (float)(p * pdf_k);
      double incl = p;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const double u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
      }
      // the previous lane's inclusive sum: non-decreasing along the row
      double ex = __shfl_up(incl, 1);
      if (lane == 0) ex = 0.0;
      c[t] = run + ex;
      run += __shfl(incl, 63);
    }
    const double m = run;
    float *crow = cl + (size_t)i * (W + 1);
    if (m > 0.0) {
      const double invm = 1.0 / m;
#pragma unroll
      for (int t = 0; t < SEG; ++t) {
        const int j = 64 * t + lane;
        if (j < W) crow[j] = (float)(c[t] * invm);
      }
    } else {
#pragma unroll
      for (int t = 0; t < SEG; ++t) {
        const int j = 64 * t + lane;
        if (j < W) crow[j] = (float)((double)j / (double)W);
      }
    }
    if (lane == 0) {
      crow[W] = 1.0f;
      rowmass[i] = m;
    }
  }
  __syncthreads();
  // marginal over rows (wavefront 0)
  if (wave == 0) {
    const int rseg = (H + 63) / 64;
    const int i0 = lane * rseg;
    double part = 0.0;
    for (int t = 0; t < rseg; ++t)
      if (i0 + t < H) part += rowmass[i0 + t];
    double c = wave_excl_scan(part, lane);
    for (int t = 0; t < rseg; ++t) {
      const int i = i0 + t;
      if (i < H) {
        ml[i] = (float)c;
        c += rowmass[i];
      }
    }
    if (lane == 0) {
      ml[H] = 1.0f;
      if (tl) *tl = S;
    }
  }
}

template <class OUT>
hipError_t launch_cdf_t(const float *density, uint32_t L, int H, int W, const OUT &o, uint32_t *err,
                        hipStream_t s) {
  const size_t lds = sizeof(double) * H;
  const int seg = (W + 63) / 64;  // W is a power of two in [4, 1024]
  switch (seg) {
    case 1: hipLaunchKernelGGL((cdf_kernel<OUT, 1>), dim3(L), dim3(CDF_THREADS), lds, s, density, H, W, o, err); break;
    case 2: hipLaunchKernelGGL((cdf_kernel<OUT, 2>), dim3(L), dim3(CDF_THREADS), lds, s, density, H, W, o, err); break;
    case 4: hipLaunchKernelGGL((cdf_kernel<OUT, 4>), dim3(L), dim3(CDF_THREADS), lds, s, density, H, W, o, err); break;
    case 8: hipLaunchKernelGGL((cdf_kernel<OUT, 8>), dim3(L), dim3(CDF_THREADS), lds, s, density, H, W, o, err); break;
    default: hipLaunchKernelGGL((cdf_kernel<OUT, 16>), dim3(L), dim3(CDF_THREADS), lds, s, density, H, W, o, err);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_build_cdf(const float *density, uint32_t L, int H, int W, float *pdf, float *marg,
                            float *cond, double *total, uint32_t *err, hipStream_t s) {
  return launch_cdf_t(density, L, H, W, BatchOut{pdf, marg, cond, total}, err, s);
}

hipError_t launch_build_cdf_desc(const float *density, const npg_leaf_desc *d, uint32_t L, int H, int W,
                                 uint32_t *err, hipStream_t s) {
  return launch_cdf_t(density, L, H, W, DescOut{d}, err, s);
}
