// Guided direction sampling by table inversion, and pdf evaluation.
//
// One thread per query.  Row and column are found by searches over the
// monotone float32 tables with exact comparisons, so a query selects exactly
// the bin the definition names: the last entry <= u.
#include <math.h>

#include "npg_internal.h"

namespace {

// largest i in [0, n-1] with t[i] <= u, for t non-decreasing with
// t[0] <= u < t[n].  The search starts at the entry a linear table would
// hold u at, gallops outwards until u is bracketed and bisects the bracket:
// for smooth tables the first probe and its neighbour share a cache line.
__device__ __forceinline__ int last_le(const float *__restrict__ t, int n, float u) {
  int g = (int)(u * (float)n);
  g = g < n - 1 ? g : n - 1;
  int lo, hi;  // t[lo] <= u < t[hi]
  if (t[g] <= u) {
    lo = g;
    for (int step = 1;; step <<= 1) {
      hi = lo + step;
      if (hi >= n) {
        hi = n;
        break;
      }
      if (t[hi] > u) break;
      lo = hi;
    }
  } else {
    hi = g;
    for (int step = 1;; step <<= 1) {
      lo = hi - step;
      if (lo <= 0) {
        lo = 0;
        break;
      }
      if (t[lo] <= u) break;
      hi = lo;
    }
  }
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (t[mid] <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void sample_kernel(
    const float *__restrict__ pdf, const float *__restrict__ marg, const float *__restrict__ cond,
    uint32_t L, int H, int W, const uint32_t *__restrict__ leaf, const float2 *__restrict__ u, uint64_t n,
    float *__restrict__ dir, float *__restrict__ pdf_out, uint32_t *__restrict__ bin_out, uint32_t *err) {
  const float below1 = __int_as_float(0x3f7fffff);
  const float two_over_h = 2.0f / (float)H;
  const float dphi = 6.283185307179586f / (float)W;
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t l = leaf[q];
    const float2 uu = u[q];
    if (l >= L || !(uu.x >= 0.0f && uu.x < 1.0f) || !(uu.y >= 0.0f && uu.y < 1.0f)) {
      const float qnan = __int_as_float(0x7fc00000);
      dir[3 * q] = qnan;
      dir[3 * q + 1] = qnan;
      dir[3 * q + 2] = qnan;
      pdf_out[q] = qnan;
      if (bin_out) bin_out[q] = 0xffffffffu;
      raise_err(err, ERR_RANGE);
      continue;
    }
    const float *M = marg + (size_t)l * (H + 1);
    const int i = last_le(M, H, uu.x);
    const float *C = cond + ((size_t)l * H + i) * (W + 1);
    const int j = last_le(C, W, uu.y);
    const float m0 = M[i], m1 = M[i + 1];
    const float c0 = C[j], c1 = C[j + 1];
    float t1 = (uu.x - m0) / (m1 - m0);
    float t2 = (uu.y - c0) / (c1 - c0);
    t1 = fminf(fmaxf(t1, 0.0f), below1);
    t2 = fminf(fmaxf(t2, 0.0f), below1);
    // -1 + 2i/H, 2i/H and 2(H-i)/H are exact; each of z, 1+z, 1-z takes
    // one rounding, so sin(theta) = sqrt((1-z)(1+z)) stays accurate at the
    // poles where 1 - z*z would cancel.
    const float z = fmaf(t1, two_over_h, fmaf((float)i, two_over_h, -1.0f));
    const float opz = fmaf(t1, two_over_h, (float)i * two_over_h);
    const float omz = fmaf(-t1, two_over_h, (float)(H - i) * two_over_h);
    const float phi = fmaf(t2, dphi, (float)j * dphi);
    float sp, cp;
    sincosf(phi, &sp, &cp);
    const float r = sqrtf(fmaxf(0.0f, omz * opz));
    dir[3 * q] = r * cp;
    dir[3 * q + 1] = r * sp;
    dir[3 * q + 2] = z;
    pdf_out[q] = pdf[(size_t)l * H * W + (size_t)i * W + j];
    if (bin_out) bin_out[q] = (uint32_t)(i * W + j);
  }
}

__global__ __launch_bounds__(256) void eval_kernel(const float2 *__restrict__ bnd, const float *__restrict__ pdf, uint32_t L, int H, int W,
                                                   const uint32_t *__restrict__ leaf,
                                                   const float *__restrict__ dir, uint64_t n,
                                                   float *__restrict__ out, uint32_t *err) {
  __shared__ float2 q4[256];
  load_quarter(bnd, W, q4);
  __syncthreads();
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t l = leaf[q];
    const float x = dir[3 * q], y = dir[3 * q + 1], z = dir[3 * q + 2];
    if (l >= L || !finite3(x, y, z)) {
      out[q] = 0.0f;
      raise_err(err, ERR_RANGE);
      continue;
    }
    const int k = z_row(z, H) * W + phi_sector(q4, x, y, W);
    out[q] = pdf[(size_t)l * H * W + k];
  }
}

size_t grid_for(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return (size_t)(b < 262144 ? b : 262144);
}

}  // namespace

hipError_t launch_sample(const npg_tables &t, const uint32_t *leaf, const float *u, uint64_t n,
                         float *dir, float *pdf, uint32_t *bin, uint32_t *err, hipStream_t s) {
  hipLaunchKernelGGL(sample_kernel, dim3(grid_for(n)), dim3(256), 0, s, t.pdf_dev, t.marg_dev, t.cond_dev,
                     t.L, t.H, t.W, leaf, reinterpret_cast<const float2 *>(u), n, dir, pdf, bin, err);
  return hipGetLastError();
}

hipError_t launch_eval(const float2 *bnd, const npg_tables &t, const uint32_t *leaf, const float *dir, uint64_t n, float *pdf,
                       uint32_t *err, hipStream_t s) {
  hipLaunchKernelGGL(eval_kernel, dim3(grid_for(n)), dim3(256), 0, s, bnd, t.pdf_dev, t.L, t.H, t.W, leaf, dir,
                     n, pdf, err);
  return hipGetLastError();
}
