// Context, error handling, scratch arena and the entry points whose work is
// a single kernel family (splat, normalise, CDF, sample, eval).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "npg_internal.h"

int npg_fail(npg_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return code;
}

int npg_set_device(npg_ctx *ctx) {
  NPG_HIP_CHECK(ctx, hipSetDevice(ctx->device));
  return NPG_OK;
}

void npg_host_boundaries(float2 out[256]) {
  // t_m = fl64(2*pi*m)/1024; c, s rounded once from binary64 cos/sin.
  for (int m = 0; m < 256; ++m) {
    const double t = (2.0 * M_PI * (double)m) / 1024.0;
    out[m] = make_float2((float)cos(t), (float)sin(t));
  }
}

int npg_device_alloc(npg_ctx *ctx, size_t bytes, void **out) {
  if (ctx->budget && ctx->held + bytes > ctx->budget)
    return npg_fail(ctx, NPG_E_BUDGET, "device allocation of %zu bytes exceeds the budget (%llu held of %llu)",
                    bytes, (unsigned long long)ctx->held, (unsigned long long)ctx->budget);
  NPG_HIP_CHECK(ctx, hipMalloc(out, bytes ? bytes : 1));
  ctx->held += bytes;
  if (ctx->held > ctx->peak) ctx->peak = ctx->held;
  return NPG_OK;
}

void npg_device_free(npg_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->held -= bytes;
}

int npg_scratch(npg_ctx *ctx, size_t bytes, hipStream_t stream, void **out) {
  bytes = npg_align(bytes, 1 << 20);
  if (bytes > ctx->scratch_bytes) {
    if (ctx->scratch) {
      // The old buffer may still be read by work queued earlier.
      NPG_HIP_CHECK(ctx, hipStreamSynchronize(ctx->scratch_stream));
      if (ctx->scratch_stream != stream) NPG_HIP_CHECK(ctx, hipStreamSynchronize(stream));
      npg_device_free(ctx, ctx->scratch, ctx->scratch_bytes);
      ctx->scratch = nullptr;
      ctx->scratch_bytes = 0;
    }
    int rc = npg_device_alloc(ctx, bytes, &ctx->scratch);
    if (rc) {
      ctx->scratch = nullptr;
      return rc;
    }
    ctx->scratch_bytes = bytes;
  }
  ctx->scratch_stream = stream;
  *out = ctx->scratch;
  return NPG_OK;
}

extern "C" {

int npg_create(npg_ctx **out, int device, uint64_t hbm_budget_bytes) {
  if (!out) return NPG_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return NPG_E_HIP;
  if (device < 0 || device >= ndev) return NPG_E_ARG;
  npg_ctx *ctx = new npg_ctx();
  ctx->device = device;
  ctx->budget = hbm_budget_bytes;
  int rc = npg_set_device(ctx);
  if (!rc) {
    // one allocation: error word (256 B) + boundary table (2 KiB)
    void *p = nullptr;
    rc = npg_device_alloc(ctx, 256 + sizeof(float2) * 256, &p);
    if (!rc) {
      ctx->err_dev = static_cast<uint32_t *>(p);
      ctx->bnd_dev = reinterpret_cast<float2 *>(static_cast<char *>(p) + 256);
      float2 tab[256];
      npg_host_boundaries(tab);
      if (hipMemset(ctx->err_dev, 0, sizeof(uint32_t)) != hipSuccess ||
          hipMemcpy(ctx->bnd_dev, tab, sizeof(tab), hipMemcpyHostToDevice) != hipSuccess)
        rc = NPG_E_HIP;
    }
  }
  if (!rc) rc = npg_noalloc_setup(ctx);
  if (rc) {
    npg_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return NPG_OK;
}

void npg_destroy(npg_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
  npg_device_free(ctx, ctx->scratch, ctx->scratch_bytes);
  npg_device_free(ctx, ctx->err_dev, 256 + sizeof(float2) * 256);
  delete ctx;
}

const char *npg_last_error(const npg_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int npg_set_option(npg_ctx *ctx, const char *name, int64_t value) {
  if (!ctx || !name) return NPG_E_ARG;
  const std::string n(name);
  if (n != "graphs" && n != "chunk_leaves" && n != "force_direct" && n != "fuse_first" &&
      n != "upsample_taps9" && n != "pool_outputs" && n != "tile_cap")
    return npg_fail(ctx, NPG_E_ARG, "unknown option '%s'", name);
  if (value < 0) return npg_fail(ctx, NPG_E_ARG, "option '%s' must be >= 0", name);
  ctx->opts[n] = value;
  return NPG_OK;
}

void npg_memory_usage(const npg_ctx *ctx, uint64_t *current, uint64_t *peak) {
  if (current) *current = ctx ? ctx->held : 0;
  if (peak) *peak = ctx ? ctx->peak : 0;
}

void npg_conv_flops(npg_ctx *ctx, double *matrix, double *vector, int reset) {
  if (matrix) *matrix = ctx ? ctx->conv_flops[0] : 0.0;
  if (vector) *vector = ctx ? ctx->conv_flops[1] : 0.0;
  if (ctx && reset) ctx->conv_flops[0] = ctx->conv_flops[1] = 0.0;
}

int npg_sync_status(npg_ctx *ctx, void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t flag = 0;
  NPG_HIP_CHECK(ctx, hipMemcpyAsync(&flag, ctx->err_dev, sizeof(flag), hipMemcpyDeviceToHost, s));
  NPG_HIP_CHECK(ctx, hipStreamSynchronize(s));
  if (flag) {
    NPG_HIP_CHECK(ctx, hipMemsetAsync(ctx->err_dev, 0, sizeof(uint32_t), s));
    NPG_HIP_CHECK(ctx, hipStreamSynchronize(s));
    return npg_fail(ctx, NPG_E_RANGE, "a kernel flagged a data-dependent range error (0x%x)", flag);
  }
  return NPG_OK;
}

int npg_bin_boundaries(int W, float *xy_out) {
  if (!pow2_in(W, 4, 1024) || !xy_out) return NPG_E_ARG;
  float2 tab[256];
  npg_host_boundaries(tab);
  const int Q = W / 4;
  for (int b = 0; b < W; ++b) {
    const int q = b / Q, r = b % Q;
    const float2 e = tab[r * (1024 / W)];
    float x, y;
    switch (q) {
      case 0: x = e.x; y = e.y; break;
      case 1: x = -e.y; y = e.x; break;
      case 2: x = -e.x; y = -e.y; break;
      default: x = e.y; y = -e.x; break;
    }
    xy_out[2 * b] = x;
    xy_out[2 * b + 1] = y;
  }
  return NPG_OK;
}

int npg_splat_histograms(npg_ctx *ctx, const float *dir_dev, const uint32_t *w_dev,
                         const uint32_t *perm_dev, const uint32_t *leaf_off_dev, uint32_t L,
                         int H, int W, uint64_t *energy_dev, uint32_t *count_dev, int accumulate,
                         void *stream) {
  if (!ctx) return NPG_E_ARG;
  if (!pow2_in(H, 4, 1024) || !pow2_in(W, 4, 1024))
    return npg_fail(ctx, NPG_E_ARG, "splat: H=%d W=%d must be powers of two in [4,1024]", H, W);
  if (L == 0) return NPG_OK;
  if (!dir_dev || !w_dev || !leaf_off_dev || !energy_dev)
    return npg_fail(ctx, NPG_E_ARG, "splat: null pointer");
  int rc = npg_set_device(ctx);
  if (rc) return rc;
  NPG_HIP_CHECK(ctx, launch_splat(ctx->bnd_dev, dir_dev, w_dev, perm_dev, leaf_off_dev, L, H, W, energy_dev,
                                  count_dev, accumulate ? 1 : 0, ctx->err_dev,
                                  static_cast<hipStream_t>(stream)));
  return NPG_OK;
}

int npg_normalize_input(npg_ctx *ctx, const uint64_t *energy_dev, uint32_t L, int H, int W,
                        float *x_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  if (!pow2_in(H, 4, 1024) || !pow2_in(W, 4, 1024))
    return npg_fail(ctx, NPG_E_ARG, "normalize: bad H=%d W=%d", H, W);
  if (L == 0) return NPG_OK;
  if (!energy_dev || !x_dev) return npg_fail(ctx, NPG_E_ARG, "normalize: null pointer");
  int rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void *scr = nullptr;
  rc = npg_scratch(ctx, sizeof(double) * (size_t)L, s, &scr);
  if (rc) return rc;
  double *tot = static_cast<double *>(scr);
  NPG_HIP_CHECK(ctx, launch_leaf_scale(energy_dev, L, H * W, tot, s));
  NPG_HIP_CHECK(ctx, launch_apply_scale(energy_dev, tot, L, H * W, x_dev, s));
  return NPG_OK;
}

int npg_build_cdf(npg_ctx *ctx, const float *density_dev, uint32_t L, int H, int W, float *pdf_dev,
                  float *marg_dev, float *cond_dev, double *total_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  if (!pow2_in(H, 4, 1024) || !pow2_in(W, 4, 1024))
    return npg_fail(ctx, NPG_E_ARG, "build_cdf: bad H=%d W=%d", H, W);
  if (L == 0) return NPG_OK;
  if (!density_dev || !pdf_dev || !marg_dev || !cond_dev)
    return npg_fail(ctx, NPG_E_ARG, "build_cdf: null pointer");
  int rc = npg_set_device(ctx);
  if (rc) return rc;
  NPG_HIP_CHECK(ctx, launch_build_cdf(density_dev, L, H, W, pdf_dev, marg_dev, cond_dev, total_dev,
                                      ctx->err_dev, static_cast<hipStream_t>(stream)));
  return NPG_OK;
}

static int check_tables(npg_ctx *ctx, const npg_tables *t, bool need_cdf) {
  if (!t) return npg_fail(ctx, NPG_E_ARG, "null tables");
  if (!pow2_in(t->H, 4, 1024) || !pow2_in(t->W, 4, 1024))
    return npg_fail(ctx, NPG_E_ARG, "tables: bad H=%d W=%d", t->H, t->W);
  if (!t->pdf_dev || (need_cdf && (!t->marg_dev || !t->cond_dev)))
    return npg_fail(ctx, NPG_E_ARG, "tables: null pointer");
  return NPG_OK;
}

int npg_sample_dirs(npg_ctx *ctx, const npg_tables *tables, const uint32_t *leaf_dev,
                    const float *u_dev, uint64_t n, float *dir_out_dev, float *pdf_out_dev,
                    uint32_t *bin_out_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = check_tables(ctx, tables, true);
  if (rc) return rc;
  if (n == 0) return NPG_OK;
  if (!leaf_dev || !u_dev || !dir_out_dev || !pdf_out_dev)
    return npg_fail(ctx, NPG_E_ARG, "sample: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  NPG_HIP_CHECK(ctx, launch_sample(*tables, leaf_dev, u_dev, n, dir_out_dev, pdf_out_dev,
                                   bin_out_dev, ctx->err_dev, static_cast<hipStream_t>(stream)));
  return NPG_OK;
}

int npg_eval_pdf(npg_ctx *ctx, const npg_tables *tables, const uint32_t *leaf_dev,
                 const float *dir_dev, uint64_t n, float *pdf_out_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = check_tables(ctx, tables, false);
  if (rc) return rc;
  if (n == 0) return NPG_OK;
  if (!leaf_dev || !dir_dev || !pdf_out_dev) return npg_fail(ctx, NPG_E_ARG, "eval: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  NPG_HIP_CHECK(ctx, launch_eval(ctx->bnd_dev, *tables, leaf_dev, dir_dev, n, pdf_out_dev, ctx->err_dev,
                                 static_cast<hipStream_t>(stream)));
  return NPG_OK;
}

int npg_mis_alpha(npg_ctx *ctx, const float *nu_b_dev, const float *nu_g_dev, const uint32_t *q_b_dev,
                  const uint32_t *q_g_dev, uint32_t L, float *alpha_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  if (L == 0) return NPG_OK;
  if (!nu_b_dev || !nu_g_dev || !q_b_dev || !q_g_dev || !alpha_dev)
    return npg_fail(ctx, NPG_E_ARG, "mis_alpha: null pointer");
  int rc = npg_set_device(ctx);
  if (rc) return rc;
  NPG_HIP_CHECK(ctx, launch_mis_alpha(nu_b_dev, nu_g_dev, q_b_dev, q_g_dev, L, alpha_dev, ctx->err_dev,
                                      static_cast<hipStream_t>(stream)));
  return NPG_OK;
}

int npg_sample_mis(npg_ctx *ctx, const npg_tables *tables, const float *alpha_dev, const uint32_t *leaf_dev,
                   const float *normal_dev, const float *u_dev, uint64_t n, float *dir_out_dev,
                   float *pdf_out_dev, uint8_t *strategy_out_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = check_tables(ctx, tables, true);
  if (rc) return rc;
  if (n == 0) return NPG_OK;
  if (!alpha_dev || !leaf_dev || !normal_dev || !u_dev || !dir_out_dev || !pdf_out_dev)
    return npg_fail(ctx, NPG_E_ARG, "sample_mis: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  NPG_HIP_CHECK(ctx, launch_sample_mis(ctx->bnd_dev, *tables, alpha_dev, leaf_dev, normal_dev, u_dev, n,
                                       dir_out_dev, pdf_out_dev, strategy_out_dev, ctx->err_dev,
                                       static_cast<hipStream_t>(stream)));
  return NPG_OK;
}

int npg_eval_pdf_mis(npg_ctx *ctx, const npg_tables *tables, const float *alpha_dev, const uint32_t *leaf_dev,
                     const float *normal_dev, const float *dir_dev, uint64_t n, float *pdf_out_dev,
                     void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = check_tables(ctx, tables, false);
  if (rc) return rc;
  if (n == 0) return NPG_OK;
  if (!alpha_dev || !leaf_dev || !normal_dev || !dir_dev || !pdf_out_dev)
    return npg_fail(ctx, NPG_E_ARG, "eval_mis: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  NPG_HIP_CHECK(ctx, launch_eval_mis(ctx->bnd_dev, *tables, alpha_dev, leaf_dev, normal_dev, dir_dev, n,
                                     pdf_out_dev, ctx->err_dev, static_cast<hipStream_t>(stream)));
  return NPG_OK;
}

}  // extern "C"
