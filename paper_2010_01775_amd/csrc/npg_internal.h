// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <atomic>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "../../include/npg.h"

// ---------------------------------------------------------------- context
struct npg_ctx {
  int device = 0;
  uint64_t budget = 0;        // 0 = unbounded
  uint64_t held = 0;          // bytes the library holds (scratch + models)
  uint64_t peak = 0;
  uint32_t *err_dev = nullptr;  // device error word (bit 0: range error)
  float2 *bnd_dev = nullptr;    // boundary-ray table, 256 entries (see bnd_ray)
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  hipStream_t scratch_stream = nullptr;  // stream that last used the scratch
  std::string last_error;
  std::map<std::string, long long> opts;          // npg_set_option
  std::map<std::string, std::vector<int>> tune;   // autotuned {chunk, tile cap per conv call}
  struct Graph {
    std::string key;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;                      // captured fused calls
  std::set<std::string> graph_seen;
  // FLOPs of the network convolutions as launched since the last reset
  // (npg_conv_flops): [0] issued on the matrix cores, [1] on the vector ALUs
  double conv_flops[2] = {0.0, 0.0};
  // device address of the library's static network scratch array on this
  // context's device (npg_reconstruct_density_noalloc), set by npg_create
  void *noalloc_scratch = nullptr;
  long long opt(const char *name, long long def) const {
    auto it = opts.find(name);
    return it == opts.end() ? def : it->second;
  }
};

// Error bits raised by kernels into ctx->err_dev.
enum : uint32_t { ERR_RANGE = 1u };

int npg_fail(npg_ctx *ctx, int code, const char *fmt, ...);
#define NPG_HIP_CHECK(ctx, expr)                                                     \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return npg_fail((ctx), NPG_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

// Scratch arena: one device buffer per context, grown on demand within the
// budget.  Growing waits for the stream that last used the old buffer.
int npg_scratch(npg_ctx *ctx, size_t bytes, hipStream_t stream, void **out);
int npg_device_alloc(npg_ctx *ctx, size_t bytes, void **out);
void npg_device_free(npg_ctx *ctx, void *p, size_t bytes);
int npg_set_device(npg_ctx *ctx);
// Looks up (once per device, with ctx's device current) the device address
// of the static scratch array of npg_reconstruct_density_noalloc and keeps it
// in ctx->noalloc_scratch.
int npg_noalloc_setup(npg_ctx *ctx);

__host__ __device__ static inline size_t npg_align(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// A kernel's LDS limit is raised on every device it runs on: true the first
// time the calling thread's current device (0..63) meets `done`, which then
// records it (a caller whose attribute call fails returns that error).
static inline bool npg_first_on_device(std::atomic<uint64_t> &done) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return true;
  const uint64_t bit = 1ull << (dev & 63);
  return !(done.fetch_or(bit) & bit);
}

// Carves consecutive 256-byte aligned pieces out of one scratch buffer.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <class T>
  T *take(size_t count) {
    T *p = reinterpret_cast<T *>(base + off);
    off += npg_align(count * sizeof(T));
    return p;
  }
};

static inline bool pow2_in(int v, int lo, int hi) {
  return v >= lo && v <= hi && (v & (v - 1)) == 0;
}

// ---------------------------------------------------------------- bin rule
// Boundary rays of the azimuth sectors.  The context holds the table
// tab[m] = (RN32(cos t), RN32(sin t)), t = fl64(2*pi*m)/1024, m = 0..255: the
// first quadrant of a 1024-column map.  A W-column map uses ray r*(1024/W)
// for its r-th ray (the binary64 angles coincide exactly because W is a power
// of two), rotated by q*90 degrees for quadrant q.  Kernels stage the W/4
// rays they need into LDS with load_quarter and index them with bnd_ray.
void npg_host_boundaries(float2 out[256]);

__device__ __forceinline__ void load_quarter(const float2 *__restrict__ tab1024, int W, float2 *q) {
  for (int r = threadIdx.x; r < (W >> 2); r += blockDim.x) q[r] = tab1024[r * (1024 / W)];
}

__device__ __forceinline__ float2 bnd_ray(const float2 *q4, int b, int W) {
  const int Q = W >> 2;                          // a power of two
  const int q = b >> (__builtin_ctz((unsigned)W) - 2);
  const float2 e = q4[b & (Q - 1)];
  // rotation by q quarter turns (negations are exact): an odd q turns
  // (x, y) into (-y, x), q >= 2 negates both
  float cx = (q & 1) ? -e.y : e.x, cy = (q & 1) ? e.x : e.y;
  if (q & 2) cx = -cx, cy = -cy;
  return make_float2(cx, cy);
}

// Sign test of cross(e, v) = e.x*y - e.y*x.  Both products of float32
// operands are exact in binary64, so the sign of their rounded difference is
// the sign of the exact value.
__device__ __forceinline__ bool left_of(float2 e, float x, float y) {
  const double a = (double)e.x * (double)y;
  const double b = (double)e.y * (double)x;
  return a - b >= 0.0;
}

// Estimate of atan2(y, x) in [-pi, pi] for (x, y) != 0: the odd polynomial of
// Abramowitz & Stegun 4.4.47 for atan on [0, 1] (absolute error <= 1e-5),
// applied to min/max of |x|, |y| and unfolded to the octant.  Callers settle
// the exact answer with exact tests; the estimate only has to be close.
__device__ __forceinline__ float atan2_est(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float t = fminf(mn * __builtin_amdgcn_rcpf(mx), 1.0f);  // in [0, 1] even for subnormal inputs
  const float t2 = t * t;
  float r = fmaf(fmaf(fmaf(fmaf(0.0208351f, t2, -0.0851330f), t2, 0.1801410f), t2, -0.3302995f), t2, 0.9998660f) * t;
  if (ay > ax) r = 1.57079632679f - r;
  if (x < 0.0f) r = 3.14159265359f - r;
  return y < 0.0f ? -r : r;
}

// Azimuth sector of (x, y): the b with cross(e_b, v) >= 0 > cross(e_{b+1}, v).
// An atan2 estimate lands within one sector of the answer (its error is far
// below the sector width 2 pi / W >= 6e-3 rad); the exact tests then settle
// it.  A bisection over all sectors backs up the (never observed) case of a
// farther estimate.
__device__ __forceinline__ int phi_sector(const float2 *q4, float x, float y, int W) {
  if (x == 0.0f && y == 0.0f) return 0;
  const float k = (float)W * 0.15915494309189535f;  // W / (2 pi)
  float f = atan2_est(y, x) * k;
  if (f < 0.0f) f += (float)W;
  int b = (int)f;
  b = b < 0 ? 0 : (b >= W ? W - 1 : b);
  const int mask = W - 1;
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    if (!left_of(bnd_ray(q4, b, W), x, y)) {
      b = (b - 1) & mask;
    } else if (left_of(bnd_ray(q4, (b + 1) & mask, W), x, y)) {
      b = (b + 1) & mask;
    } else {
      return b;
    }
  }
  // Quadrant from the axis rays (exact), then bisection on the half-plane
  // test inside it: left_of(e_b) is true for b <= answer, false after.
  int q;
  if (y >= 0.0f && x > 0.0f) q = 0;
  else if (x <= 0.0f && y > 0.0f) q = 1;
  else if (y <= 0.0f && x < 0.0f) q = 2;
  else q = 3;
  int lo = q * (W >> 2), hi = lo + (W >> 2) - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (left_of(bnd_ray(q4, mid, W), x, y)) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Row of z: #{b in 1..H-1 : z >= -1 + 2b/H}.  The boundaries are exact in
// float32 (H is a power of two <= 1024), so two corrections of a float
// estimate give the exact count.
__device__ __forceinline__ int z_row(float z, int H) {
  float t = (z + 1.0f) * (0.5f * (float)H);
  int iz = (int)floorf(fminf(fmaxf(t, 0.0f), (float)(H - 1)));
  // boundary b is -1 + b * (2 / H); 2 / H is a power of two, so the product
  // is the exact quotient b / (H / 2)
  const float ih = 2.0f / (float)H;
  if (iz > 0 && z < -1.0f + (float)iz * ih) --iz;
  if (iz > 0 && z < -1.0f + (float)iz * ih) --iz;
  if (iz < H - 1 && z >= -1.0f + (float)(iz + 1) * ih) ++iz;
  if (iz < H - 1 && z >= -1.0f + (float)(iz + 1) * ih) ++iz;
  return iz;
}

__device__ __forceinline__ bool finite3(float x, float y, float z) {
  return isfinite(x) && isfinite(y) && isfinite(z);
}

__device__ __forceinline__ void raise_err(uint32_t *err, uint32_t bit) {
  atomicOr(err, bit);
}

// Per-leaf descriptor of a serving batch: the leaf's photons (a window of a
// request's arrays) and where its tables go.
struct npg_leaf_desc {
  const float *dir;
  const uint32_t *w;
  uint32_t begin, count;
  float *pdf, *marg, *cond;
  double *total;
};

// ---------------------------------------------------------------- launchers
// Each returns a hipError_t from the launch.
hipError_t launch_splat(const float2 *bnd, const float *dir, const uint32_t *w, const uint32_t *perm,
                        const uint32_t *off, uint32_t L, int H, int W, uint64_t *energy,
                        uint32_t *count, int accumulate, uint32_t *err, hipStream_t s);
// true if the network's pooling levels divide an H x W map
bool npg_model_fits(const npg_model *m, int H, int W);
bool npg_model_fp8_ready(const npg_model *m);
int npg_model_in_channels(const npg_model *m);
hipError_t launch_splat_desc(const float2 *bnd, const npg_leaf_desc *d, uint32_t L, int H, int W,
                             uint64_t *energy, uint32_t *err, hipStream_t s);
hipError_t launch_build_cdf_desc(const float *density, const npg_leaf_desc *d, uint32_t L, int H, int W,
                                 uint32_t *err, hipStream_t s);
hipError_t launch_leaf_scale(const uint64_t *energy, uint32_t L, int HW, double *scale,
                             hipStream_t s);
hipError_t launch_apply_scale(const uint64_t *energy, const double *scale, uint32_t L, int HW,
                              float *x, hipStream_t s);
hipError_t launch_build_cdf(const float *density, uint32_t L, int H, int W, float *pdf,
                            float *marg, float *cond, double *total, uint32_t *err,
                            hipStream_t s);
hipError_t launch_sample(const npg_tables &t, const uint32_t *leaf, const float *u, uint64_t n,
                         float *dir, float *pdf, uint32_t *bin, uint32_t *err, hipStream_t s);
hipError_t launch_eval(const float2 *bnd, const npg_tables &t, const uint32_t *leaf, const float *dir, uint64_t n,
                       float *pdf, uint32_t *err, hipStream_t s);
hipError_t launch_mis_alpha(const float *nu_b, const float *nu_g, const uint32_t *q_b, const uint32_t *q_g,
                            uint32_t L, float *alpha, uint32_t *err, hipStream_t s);
hipError_t launch_sample_mis(const float2 *bnd, const npg_tables &t, const float *alpha, const uint32_t *leaf,
                             const float *normal, const float *u, uint64_t n, float *dir, float *pdf,
                             uint8_t *strat, uint32_t *err, hipStream_t s);
hipError_t launch_eval_mis(const float2 *bnd, const npg_tables &t, const float *alpha, const uint32_t *leaf,
                           const float *normal, const float *dir, uint64_t n, float *pdf, uint32_t *err,
                           hipStream_t s);

// Exclusive scan of n u32 into out[0..n] (out[n] = total); tmp holds
// npg_scan_tmp_words(n) words.
size_t npg_scan_tmp_words(uint64_t n);
hipError_t npg_scan_u32(const uint32_t *in, uint64_t n, uint32_t *out, uint32_t *tmp, hipStream_t s);
// Stable LSD radix sort (8-bit digits) of n (key, value) pairs on the low
// `bits` (1..32) bits of the keys; vals_in == nullptr: the values are the
// item indices.  The sorted pairs go to keys_out / vals_out (distinct from
// the inputs); work holds npg_radix_work_bytes(n) bytes.
size_t npg_radix_work_bytes(uint64_t n);
hipError_t npg_radix_sort(const uint32_t *keys_in, const uint32_t *vals_in, uint64_t n, int bits,
                          uint32_t *keys_out, uint32_t *vals_out, void *work, hipStream_t s);
