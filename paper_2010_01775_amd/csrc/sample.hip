// Guided direction sampling by table inversion, and pdf evaluation.
//
// One thread per query.  Row and column are found by searches over the
// monotone float32 tables with exact comparisons, so a query selects exactly
// the bin the definition names: the last entry <= u.
#include <math.h>

#include "npg_internal.h"

namespace {

// Eight table entries t[a .. a+m] (m = 7, or fewer on short rows) around
// entry g, loaded in one memory round trip.  Rows of at least 16 entries load
// a 16-byte aligned window as two 16-byte pieces (it starts 3 to 6 entries
// below g and is moved by 4 entries to stay inside the row); shorter rows
// load eight clamped single entries.  A load instruction whose 64 lanes hit
// 64 different lines costs the same at any width, so the wide loads quarter
// that cost.
__device__ __forceinline__ void load_window(const float *__restrict__ t, int n, int g, int *a_out, int *m_out,
                                            float (&w)[8]) {
  int a, m;
  if (n >= 15) {
    const uintptr_t t0 = reinterpret_cast<uintptr_t>(t);
    a = (int)(((intptr_t)((t0 + 4 * (uintptr_t)(g - 3)) & ~(uintptr_t)15) - (intptr_t)t0) / 4);
    a = a < 0 ? a + 4 : a;
    a = a < 0 ? a + 4 : a;
    a = a + 7 > n ? a - 4 : a;
    m = 7;
    const float4 *p = reinterpret_cast<const float4 *>(t + a);
    const float4 v0 = p[0], v1 = p[1];
    w[0] = v0.x, w[1] = v0.y, w[2] = v0.z, w[3] = v0.w, w[4] = v1.x, w[5] = v1.y, w[6] = v1.z, w[7] = v1.w;
  } else {
    a = g - 3;
    a = a > n - 7 ? n - 7 : a;
    a = a < 0 ? 0 : a;
    m = n - a < 7 ? n - a : 7;
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = t[a + (k < m ? k : m)];
  }
  *a_out = a;
  *m_out = m;
}

// largest i in [0, n-1] with t[i] <= u, for t non-decreasing with t[0] = 0
// <= u < t[n] = 1 (as build_cdf writes every row); *tl = t[i], *th =
// t[i+1].  The first window is placed where a linear table would hold u,
// up to three more (while none brackets u) by linear interpolation inside
// the bracket [lo, hi] the previous ones left, with its end values; each
// window settles the search when it brackets u, else narrows the bracket,
// which bisection finishes.  (On the clustered workload's tables the first
// window brackets about a third of the searches and the second most of the
// rest, where galloping outwards from the first window took several
// dependent loads: 1e8 samples 10.4 -> 7.6 ms.)  The answer is that of
// plain bisection.
__device__ __forceinline__ int last_le(const float *__restrict__ t, int n, float u, float *tl, float *th) {
  int lo = 0, hi = n;           // t[lo] <= u < t[hi]
  float tlo = 0.0f, thi = 1.0f;  // t[lo], t[hi]
  int g = (int)(u * (float)n);
  g = g < n - 1 ? g : n - 1;
#pragma unroll 1
  for (int attempt = 0; attempt < 4 && hi - lo > 1; ++attempt) {
    int a, m;
    float w[8];
    load_window(t, n, g, &a, &m, w);
    if (w[0] <= u && u < w[m]) {
      int c = 0;  // entries t[a+1 .. a+m-1] that are <= u
#pragma unroll
      for (int k = 1; k < 7; ++k) c += (k < m && w[k] <= u) ? 1 : 0;
      float lo_v = w[0], hi_v = w[1];
#pragma unroll
      for (int k = 1; k < 7; ++k)
        if (k == c) {
          lo_v = w[k];
          hi_v = w[k + 1];
        }
      *tl = lo_v;
      *th = hi_v;
      return a + c;
    }
    if (w[m] <= u) {  // the bracket lies right of the window
      if (a + m > lo) {
        lo = a + m;
        tlo = w[m];
      }
    } else if (a < hi) {  // left of it: u < t[a]
      hi = a;
      thi = w[0];
    }
    // next guess: linear inside the bracket
    const float f = thi > tlo ? (u - tlo) / (thi - tlo) : 0.0f;
    g = lo + (int)(f * (float)(hi - lo));
    g = g < lo ? lo : g;
    g = g > hi - 1 ? hi - 1 : g;
  }
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    const float v = t[mid];
    if (v <= u) {
      lo = mid;
      tlo = v;
    } else {
      hi = mid;
      thi = v;
    }
  }
  *tl = tlo;
  *th = thi;
  return lo;
}

// The guided sample of leaf l from (u1, u2): direction, the table pdf of the
// sampled bin and the bin (the leaf and the uniforms are valid).
__device__ __forceinline__ void guided_sample(const float *__restrict__ pdf, const float *__restrict__ marg,
                                              const float *__restrict__ cond, uint32_t l, int H, int W,
                                              float u1, float u2, float *d, float *p, uint32_t *bin) {
  const float below1 = __int_as_float(0x3f7fffff);
  const float two_over_h = 2.0f / (float)H;
  const float dphi = 6.283185307179586f / (float)W;
  const float *M = marg + (size_t)l * (H + 1);
  float m0, m1, c0, c1;
  const int i = last_le(M, H, u1, &m0, &m1);
  const float *C = cond + ((size_t)l * H + i) * (W + 1);
  const int j = last_le(C, W, u2, &c0, &c1);
  float t1 = (u1 - m0) / (m1 - m0);
  float t2 = (u2 - c0) / (c1 - c0);
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
  d[0] = r * cp;
  d[1] = r * sp;
  d[2] = z;
  *p = pdf[(size_t)l * H * W + (size_t)i * W + j];
  *bin = (uint32_t)(i * W + j);
}

// One query per lane, 256 consecutive queries per workgroup and iteration.
// The block's directions (3 KiB, contiguous in dir) are staged in LDS and
// written as 16-byte pieces; pdf and bin are written one lane each
// (coalesced 4-byte pieces).
__global__ __launch_bounds__(256) void sample_kernel(
    const float *__restrict__ pdf, const float *__restrict__ marg, const float *__restrict__ cond,
    uint32_t L, int H, int W, const uint32_t *__restrict__ leaf, const float2 *__restrict__ u, uint64_t n,
    float *__restrict__ dir, float *__restrict__ pdf_out, uint32_t *__restrict__ bin_out, uint32_t *err) {
  __shared__ float4 sdir[192];  // 256 directions of 3 floats
  float *sd = reinterpret_cast<float *>(sdir);
  const int t = (int)threadIdx.x;
  const bool dir16 = (reinterpret_cast<uintptr_t>(dir) & 15) == 0;
  for (uint64_t base = (uint64_t)blockIdx.x * 256; base < n; base += (uint64_t)gridDim.x * 256) {
    const uint64_t q = base + (uint64_t)t;
    float d[3] = {0.0f, 0.0f, 0.0f}, p = 0.0f;
    uint32_t b = 0;
    if (q < n) {
      const uint32_t l = leaf[q];
      const float2 uu = u[q];
      if (l >= L || !(uu.x >= 0.0f && uu.x < 1.0f) || !(uu.y >= 0.0f && uu.y < 1.0f)) {
        const float qnan = __int_as_float(0x7fc00000);
        d[0] = d[1] = d[2] = p = qnan;
        b = 0xffffffffu;
        raise_err(err, ERR_RANGE);
      } else {
        guided_sample(pdf, marg, cond, l, H, W, uu.x, uu.y, d, &p, &b);
      }
      pdf_out[q] = p;
      if (bin_out) bin_out[q] = b;
    }
    sd[3 * t] = d[0];
    sd[3 * t + 1] = d[1];
    sd[3 * t + 2] = d[2];
    __syncthreads();
    const uint64_t nb = n - base < 256 ? n - base : 256;
    float *dst = dir + 3 * base;  // 16-byte aligned when dir is (3 * 256 * 4 bytes per block)
    if (nb == 256 && dir16) {
      if (t < 192) reinterpret_cast<float4 *>(dst)[t] = sdir[t];
    } else {
      for (int k = t; k < 3 * (int)nb; k += 256) dst[k] = sd[k];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- one-sample MIS
constexpr float INV_PI = 0.3183098861837907f;

// alpha_j from the path statistics: FP64 quotient of the two averages once
// both strategies have MIS_MIN bounces, clamped to [0.2, 0.8]
constexpr uint32_t MIS_MIN = 50;
__global__ void mis_alpha_kernel(const float *__restrict__ nu_b, const float *__restrict__ nu_g,
                                 const uint32_t *__restrict__ q_b, const uint32_t *__restrict__ q_g, uint32_t L,
                                 float *__restrict__ alpha, uint32_t *err) {
  for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < L; l += gridDim.x * blockDim.x) {
    const double nb = nu_b[l], ng = nu_g[l];
    const uint32_t qb = q_b[l], qg = q_g[l];
    if (!(nb >= 0.0 && ng >= 0.0 && isfinite(nb) && isfinite(ng))) {
      alpha[l] = 0.5f;
      raise_err(err, ERR_RANGE);
      continue;
    }
    double a = 0.5;
    if (qb >= MIS_MIN && qg >= MIS_MIN) {
      const double mb = nb / (double)qb, mg = ng / (double)qg;
      if (mb + mg > 0.0) a = mb / (mb + mg);
    }
    alpha[l] = (float)fmin(fmax(a, 0.2), 0.8);
  }
}

// Cosine-lobe direction about the unit normal (nx, ny, nz) from (u1, u2):
// disk point (sqrt(u1), 2 pi u2) lifted to the hemisphere, in the frame of
// Duff et al. 2017 (sign of nz with +0 counted as positive)
__device__ __forceinline__ void cosine_sample(float nx, float ny, float nz, float u1, float u2, float *w) {
  const float sg = nz >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sg + nz);
  const float b = nx * ny * a;
  const float tx = 1.0f + sg * nx * nx * a, ty = sg * b, tz = -sg * nx;
  const float bx = b, by = sg + ny * ny * a, bz = -ny;
  const float r = sqrtf(u1);
  float sp, cp;
  sincosf(6.283185307179586f * u2, &sp, &cp);
  const float h = sqrtf(fmaxf(0.0f, 1.0f - u1));
  const float x = r * cp, y = r * sp;
  w[0] = x * tx + y * bx + h * nx;
  w[1] = x * ty + y * by + h * ny;
  w[2] = x * tz + y * bz + h * nz;
}

// The mixture a p_BSDF(w) + (1 - a) g, spelled out with explicit fused
// multiply-adds so that sampling and evaluation round it identically
// (contraction left to the compiler could differ between the two kernels).
__device__ __forceinline__ float mis_mixture(float a, float nx, float ny, float nz, const float *w, float g) {
  const float c = fmaf(nz, w[2], fmaf(ny, w[1], nx * w[0]));
  const float pb = fmaxf(0.0f, c) * INV_PI;
  return fmaf(a, pb, (1.0f - a) * g);
}

__global__ __launch_bounds__(256) void sample_mis_kernel(
    const float2 *__restrict__ bnd, const float *__restrict__ pdf, const float *__restrict__ marg,
    const float *__restrict__ cond, uint32_t L, int H, int W, const float *__restrict__ alpha,
    const uint32_t *__restrict__ leaf, const float *__restrict__ normal, const float *__restrict__ u, uint64_t n,
    float *__restrict__ dir, float *__restrict__ pdf_out, uint8_t *__restrict__ strat, uint32_t *err) {
  __shared__ float2 q4[256];
  load_quarter(bnd, W, q4);
  __syncthreads();
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t l = leaf[q];
    const float u0 = u[3 * q], u1 = u[3 * q + 1], u2 = u[3 * q + 2];
    const float nx = normal[3 * q], ny = normal[3 * q + 1], nz = normal[3 * q + 2];
    if (l >= L || !(u0 >= 0.0f && u0 < 1.0f) || !(u1 >= 0.0f && u1 < 1.0f) || !(u2 >= 0.0f && u2 < 1.0f) ||
        !finite3(nx, ny, nz)) {
      const float qnan = __int_as_float(0x7fc00000);
      dir[3 * q] = qnan;
      dir[3 * q + 1] = qnan;
      dir[3 * q + 2] = qnan;
      pdf_out[q] = qnan;
      if (strat) strat[q] = 0;
      raise_err(err, ERR_RANGE);
      continue;
    }
    const float a = alpha[l];
    float w[3], g;
    const bool bsdf = u0 < a;
    if (bsdf) {
      cosine_sample(nx, ny, nz, u1, u2, w);
      const int k = z_row(w[2], H) * W + phi_sector(q4, w[0], w[1], W);
      g = pdf[(size_t)l * H * W + k];
    } else {
      uint32_t b;
      guided_sample(pdf, marg, cond, l, H, W, u1, u2, w, &g, &b);
    }
    dir[3 * q] = w[0];
    dir[3 * q + 1] = w[1];
    dir[3 * q + 2] = w[2];
    pdf_out[q] = mis_mixture(a, nx, ny, nz, w, g);
    if (strat) strat[q] = bsdf ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void eval_mis_kernel(const float2 *__restrict__ bnd, const float *__restrict__ pdf,
                                                       uint32_t L, int H, int W, const float *__restrict__ alpha,
                                                       const uint32_t *__restrict__ leaf,
                                                       const float *__restrict__ normal,
                                                       const float *__restrict__ dir, uint64_t n,
                                                       float *__restrict__ out, uint32_t *err) {
  __shared__ float2 q4[256];
  load_quarter(bnd, W, q4);
  __syncthreads();
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t l = leaf[q];
    const float w[3] = {dir[3 * q], dir[3 * q + 1], dir[3 * q + 2]};
    const float nx = normal[3 * q], ny = normal[3 * q + 1], nz = normal[3 * q + 2];
    if (l >= L || !finite3(w[0], w[1], w[2]) || !finite3(nx, ny, nz)) {
      out[q] = 0.0f;
      raise_err(err, ERR_RANGE);
      continue;
    }
    const float a = alpha[l];
    const int k = z_row(w[2], H) * W + phi_sector(q4, w[0], w[1], W);
    out[q] = mis_mixture(a, nx, ny, nz, w, pdf[(size_t)l * H * W + k]);
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

hipError_t launch_mis_alpha(const float *nu_b, const float *nu_g, const uint32_t *q_b, const uint32_t *q_g,
                            uint32_t L, float *alpha, uint32_t *err, hipStream_t s) {
  hipLaunchKernelGGL(mis_alpha_kernel, dim3(grid_for(L)), dim3(256), 0, s, nu_b, nu_g, q_b, q_g, L, alpha, err);
  return hipGetLastError();
}

hipError_t launch_sample_mis(const float2 *bnd, const npg_tables &t, const float *alpha, const uint32_t *leaf,
                             const float *normal, const float *u, uint64_t n, float *dir, float *pdf,
                             uint8_t *strat, uint32_t *err, hipStream_t s) {
  hipLaunchKernelGGL(sample_mis_kernel, dim3(grid_for(n)), dim3(256), 0, s, bnd, t.pdf_dev, t.marg_dev, t.cond_dev,
                     t.L, t.H, t.W, alpha, leaf, normal, u, n, dir, pdf, strat, err);
  return hipGetLastError();
}

hipError_t launch_eval_mis(const float2 *bnd, const npg_tables &t, const float *alpha, const uint32_t *leaf,
                           const float *normal, const float *dir, uint64_t n, float *pdf, uint32_t *err,
                           hipStream_t s) {
  hipLaunchKernelGGL(eval_mis_kernel, dim3(grid_for(n)), dim3(256), 0, s, bnd, t.pdf_dev, t.L, t.H, t.W, alpha, leaf,
                     normal, dir, n, pdf, err);
  return hipGetLastError();
}

hipError_t launch_eval(const float2 *bnd, const npg_tables &t, const uint32_t *leaf, const float *dir, uint64_t n, float *pdf,
                       uint32_t *err, hipStream_t s) {
  hipLaunchKernelGGL(eval_kernel, dim3(grid_for(n)), dim3(256), 0, s, bnd, t.pdf_dev, t.L, t.H, t.W, leaf, dir,
                     n, pdf, err);
  return hipGetLastError();
}
