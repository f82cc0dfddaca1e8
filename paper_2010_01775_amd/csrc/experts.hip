// Mixture of experts by leaf photon count (Sec. 8, Implementation, training:
// five networks, each trained for one range of photons per voxel).
//
// route:   one workgroup computes every leaf's expert from its photon count
//          and writes, per expert, the leaves in ascending order (a stable
//          counting sort: per-thread counts, block scans, per-thread writes);
// gather:  each expert's energy maps are copied into a contiguous batch;
// network: npg_reconstruct_density with that expert's model on the batch;
// scatter: the batch's densities are copied back to their leaves.
// A leaf's density does not depend on the batch it runs in, so the result
// equals running every leaf through its expert alone.
#include "npg_internal.h"

namespace {

constexpr int MAX_EXPERTS = 8;
constexpr int ROUTE_THREADS = 1024;

struct Bounds {
  uint32_t b[MAX_EXPERTS - 1];
  int n;  // number of bounds (experts - 1)
};

__device__ __forceinline__ int expert_of(uint32_t photons, const Bounds &bd) {
  int e = 0;
#pragma unroll
  for (int k = 0; k < MAX_EXPERTS - 1; ++k)
    if (k < bd.n && bd.b[k] <= photons) ++e;
  return e;
}

// start[e] = first list slot of expert e (start[n_experts] = L); list holds
// the leaves of expert 0, then expert 1, ..., each in ascending order.
__global__ __launch_bounds__(ROUTE_THREADS) void route_kernel(const uint32_t *__restrict__ off, uint32_t L,
                                                              Bounds bd, uint32_t *__restrict__ list,
                                                              uint32_t *__restrict__ start) {
  __shared__ uint32_t wsum[MAX_EXPERTS][ROUTE_THREADS / 64];
  __shared__ uint32_t base_e[MAX_EXPERTS + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ne = bd.n + 1;
  const uint32_t per = (L + ROUTE_THREADS - 1) / ROUTE_THREADS;
  const uint32_t l0 = min(L, (uint32_t)tid * per), l1 = min(L, l0 + per);
  uint32_t cnt[MAX_EXPERTS];
#pragma unroll
  for (int e = 0; e < MAX_EXPERTS; ++e) cnt[e] = 0;
  for (uint32_t l = l0; l < l1; ++l) {
    const int e = expert_of(off[l + 1] - off[l], bd);
#pragma unroll
    for (int k = 0; k < MAX_EXPERTS; ++k) cnt[k] += (k == e) ? 1u : 0u;
  }
  // exclusive prefix of each expert's counts over the threads
  uint32_t pre[MAX_EXPERTS];
#pragma unroll
  for (int e = 0; e < MAX_EXPERTS; ++e) {
    uint32_t incl = cnt[e];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    pre[e] = incl - cnt[e];
    if (lane == 63) wsum[e][wave] = incl;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int e = 0; e < ne; ++e) {
      base_e[e] = run;
      for (int w = 0; w < ROUTE_THREADS / 64; ++w) run += wsum[e][w];
    }
    base_e[ne] = run;
    for (int e = 0; e <= ne; ++e) start[e] = base_e[e];
  }
  __syncthreads();
  uint32_t pos[MAX_EXPERTS];
#pragma unroll
  for (int e = 0; e < MAX_EXPERTS; ++e) {
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[e][w];
    pos[e] = (e < ne ? base_e[e] : 0u) + before + pre[e];
  }
  for (uint32_t l = l0; l < l1; ++l) {
    const int e = expert_of(off[l + 1] - off[l], bd);
    uint32_t p = 0;
#pragma unroll
    for (int k = 0; k < MAX_EXPERTS; ++k)
      if (k == e) p = pos[k]++;
    list[p] = l;
  }
}

// dst[i] = src[idx[i]] (gather, idx_dst == nullptr) or dst[idx[i]] = src[i]
// (scatter, idx_src == nullptr), for maps of `words` 16-byte pieces; maps
// along y, pieces along x
__global__ void move_maps_kernel(const uint4 *__restrict__ src, const uint32_t *__restrict__ idx_src,
                                 uint4 *__restrict__ dst, const uint32_t *__restrict__ idx_dst, uint32_t n,
                                 uint32_t words) {
  for (uint32_t i = blockIdx.y; i < n; i += gridDim.y) {
    const uint64_t si = idx_src ? idx_src[i] : i, di = idx_dst ? idx_dst[i] : i;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < words; k += gridDim.x * blockDim.x)
      dst[di * words + k] = src[si * words + k];
  }
}

dim3 grid_for(uint32_t n, uint32_t words) {
  return dim3(std::min<uint32_t>((words + 255) / 256, 64), std::min<uint32_t>(n, 65535));
}

}  // namespace

extern "C" int npg_reconstruct_experts(npg_ctx *ctx, const npg_model *const *models, int n_experts,
                                       const uint32_t *bounds, const uint32_t *leaf_off_dev,
                                       const uint64_t *energy_dev, uint32_t L, int H, int W,
                                       npg_precision precision, float *density_dev, uint32_t *counts_out,
                                       void *stream) {
  if (!ctx) return NPG_E_ARG;
  if (!models || n_experts < 1 || n_experts > MAX_EXPERTS)
    return npg_fail(ctx, NPG_E_ARG, "experts: n_experts %d outside [1, %d]", n_experts, MAX_EXPERTS);
  if (n_experts > 1 && !bounds) return npg_fail(ctx, NPG_E_ARG, "experts: null bounds");
  Bounds bd{};
  bd.n = n_experts - 1;
  for (int k = 0; k < bd.n; ++k) {
    bd.b[k] = bounds[k];
    if (k > 0 && bounds[k] <= bounds[k - 1])
      return npg_fail(ctx, NPG_E_ARG, "experts: bounds must increase strictly");
  }
  for (int e = 0; e < n_experts; ++e)
    if (!models[e]) return npg_fail(ctx, NPG_E_ARG, "experts: null model %d", e);
  if (!pow2_in(H, 4, 1024) || !pow2_in(W, 4, 1024))
    return npg_fail(ctx, NPG_E_ARG, "experts: H, W must be powers of two in [4, 1024]");
  if (counts_out)
    for (int e = 0; e < n_experts; ++e) counts_out[e] = 0;
  if (L == 0) return NPG_OK;
  if (!leaf_off_dev || !energy_dev || !density_dev) return npg_fail(ctx, NPG_E_ARG, "experts: null pointer");
  if (((uintptr_t)energy_dev | (uintptr_t)density_dev) & 15)
    return npg_fail(ctx, NPG_E_ARG, "experts: energy and density must be 16-byte aligned");
  int rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t HW = (size_t)H * W;
  // gather batches of at most G leaves: 12 bytes per bin (energy + density)
  size_t G = std::min<size_t>(L, std::max<size_t>(1, ((size_t)1 << 30) / (HW * 12)));
  if (ctx->budget) {
    const uint64_t free_b = ctx->budget > ctx->held ? ctx->budget - ctx->held : 0;
    G = std::min<size_t>(G, std::max<size_t>(1, free_b / 4 / (HW * 12)));
  }
  const int64_t opt_chunk = ctx->opt("chunk_leaves", 0);
  if (opt_chunk > 0) G = std::min<size_t>(G, (size_t)opt_chunk);
  const size_t bytes = npg_align(sizeof(uint32_t) * ((size_t)L + MAX_EXPERTS + 1)) +
                       npg_align(HW * sizeof(uint64_t) * G) + npg_align(HW * sizeof(float) * G);
  void *buf = nullptr;
  rc = npg_device_alloc(ctx, bytes, &buf);
  if (rc) return rc;
  Carver cv(buf);
  uint32_t *list = cv.take<uint32_t>(L);
  uint32_t *start = cv.take<uint32_t>(MAX_EXPERTS + 1);
  uint64_t *eg = cv.take<uint64_t>(HW * G);
  float *dg = cv.take<float>(HW * G);
  uint32_t st[MAX_EXPERTS + 1] = {0};
  auto finish = [&](int code) {
    (void)hipStreamSynchronize(s);  // the buffers may still be read by queued work
    npg_device_free(ctx, buf, bytes);
    return code;
  };
  hipLaunchKernelGGL(route_kernel, dim3(1), dim3(ROUTE_THREADS), 0, s, leaf_off_dev, L, bd, list, start);
  if (hipGetLastError() != hipSuccess) return finish(npg_fail(ctx, NPG_E_HIP, "experts: route launch"));
  if (hipMemcpyAsync(st, start, sizeof(uint32_t) * (n_experts + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return finish(npg_fail(ctx, NPG_E_HIP, "experts: reading the expert sizes"));
  if (st[n_experts] != L) return finish(npg_fail(ctx, NPG_E_HIP, "experts: routing lost leaves"));
  for (int e = 0; e < n_experts; ++e) {
    if (counts_out) counts_out[e] = st[e + 1] - st[e];
    for (uint32_t b0 = st[e]; b0 < st[e + 1]; b0 += (uint32_t)G) {
      const uint32_t n = (uint32_t)std::min<size_t>(G, st[e + 1] - b0);
      const uint32_t ew = (uint32_t)(HW * sizeof(uint64_t) / 16), dw = (uint32_t)(HW * sizeof(float) / 16);
      hipLaunchKernelGGL(move_maps_kernel, grid_for(n, ew), dim3(256), 0, s,
                         reinterpret_cast<const uint4 *>(energy_dev), list + b0, reinterpret_cast<uint4 *>(eg),
                         nullptr, n, ew);
      if (hipGetLastError() != hipSuccess) return finish(npg_fail(ctx, NPG_E_HIP, "experts: gather launch"));
      rc = npg_reconstruct_density(ctx, models[e], eg, nullptr, n, H, W, precision, dg, stream);
      if (rc) return finish(rc);
      hipLaunchKernelGGL(move_maps_kernel, grid_for(n, dw), dim3(256), 0, s,
                         reinterpret_cast<const uint4 *>(dg), nullptr, reinterpret_cast<uint4 *>(density_dev),
                         list + b0, n, dw);
      if (hipGetLastError() != hipSuccess) return finish(npg_fail(ctx, NPG_E_HIP, "experts: scatter launch"));
    }
  }
  return finish(NPG_OK);
}
