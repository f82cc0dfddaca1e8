// Serving: continuous batching of reconstruction and sampling requests.
//
// A scheduler thread owns `n_slots` device streams, each with its own
// context (scratch).  Reconstruction requests (photons already in device
// memory, per-leaf photon windows given on the host) wait in a FIFO.
// Whenever a slot is free, the scheduler takes the oldest waiting request and
// merges every later waiting request of the same map size into the same
// batch, up to `max_batch_leaves` leaves and as long as their tables fit in
// the table arena; one batch runs as one chain of kernels (splat -> network
// -> CDF) over the leaves of all its requests, addressed through per-leaf
// descriptors.  Tables stay resident in the arena until the client releases
// the request, so later sampling requests read them directly.  Sampling
// requests run on any free slot after the event of their reconstruction.
// Requests admitted while others run overlap on the device (one stream per
// slot).  A leaf's result does not depend on the batch it lands in: every
// kernel computes each leaf independently, in the same order.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>

#include "npg_internal.h"
#include "serve_core.h"

int npg_run_desc_batch(npg_ctx *ctx, const npg_model *m, npg_precision prec, const npg_leaf_desc *d_dev,
                       uint32_t L, int H, int W, hipStream_t s);

namespace {

using Clock = std::chrono::steady_clock;
using npg_serve_core::Req;

double now_us() {
  return std::chrono::duration<double, std::micro>(Clock::now().time_since_epoch()).count();
}

struct Slot {
  npg_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  npg_leaf_desc *desc_dev = nullptr;
  npg_leaf_desc *desc_host = nullptr;  // pinned
  size_t desc_cap = 0;
};

// The device side of the server: one stream, context and completion event
// per slot, and the event after which each reconstruction's tables are ready.
struct HipExec {
  const npg_model *model = nullptr;
  npg_precision precision = NPG_FP32;
  std::vector<Slot> slots;
  std::map<uint64_t, hipEvent_t> ready;

  double now_us() const { return ::now_us(); }
  const char *slot_error(int si) const { return slots[si].ctx->last_error.c_str(); }

  int query(int si) {
    const hipError_t q = hipEventQuery(slots[si].done);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) {
      slots[si].ctx->last_error = hipGetErrorString(q);
      return -1;
    }
    return 1;
  }

  void forget(Req &r) {
    auto it = ready.find(r.id);
    if (it != ready.end()) {
      (void)hipEventDestroy(it->second);
      ready.erase(it);
    }
  }

  int launch_sample(int si, Req &r, const Req &rc) {
    Slot &sl = slots[si];
    auto ev = ready.find(rc.id);
    if (ev != ready.end()) NPG_HIP_CHECK(sl.ctx, hipStreamWaitEvent(sl.stream, ev->second, 0));
    npg_tables t{rc.pdf, rc.marg, rc.cond, rc.total, rc.L, rc.H, rc.W};
    NPG_HIP_CHECK(sl.ctx,
                  ::launch_sample(t, r.leaf, r.u, r.n, r.dir_out, r.pdf_out, nullptr, sl.ctx->err_dev, sl.stream));
    NPG_HIP_CHECK(sl.ctx, hipEventRecord(sl.done, sl.stream));
    return NPG_OK;
  }

  // one chain of kernels (splat -> network -> CDF) over the leaves of every
  // request of the batch, addressed through per-leaf descriptors
  int launch_recon(int si, const std::vector<Req *> &batch, uint32_t L) {
    Slot &sl = slots[si];
    if (L > sl.desc_cap) {
      if (sl.desc_dev) (void)hipFree(sl.desc_dev);
      if (sl.desc_host) (void)hipHostFree(sl.desc_host);
      sl.desc_dev = nullptr;
      sl.desc_host = nullptr;
      sl.desc_cap = 0;
      const size_t cap = std::max<size_t>(L, 4096);
      NPG_HIP_CHECK(sl.ctx, hipMalloc(&sl.desc_dev, cap * sizeof(npg_leaf_desc)));
      NPG_HIP_CHECK(sl.ctx, hipHostMalloc(&sl.desc_host, cap * sizeof(npg_leaf_desc)));
      sl.desc_cap = cap;
    }
    uint32_t k = 0;
    for (const Req *r : batch) {
      const size_t HW = (size_t)r->H * r->W;
      for (uint32_t l = 0; l < r->L; ++l, ++k) {
        npg_leaf_desc &d = sl.desc_host[k];
        d.dir = r->dir;
        d.w = r->w;
        d.begin = r->beg[l];
        d.count = r->cnt[l];
        d.pdf = r->pdf + l * HW;
        d.marg = r->marg + (size_t)l * (r->H + 1);
        d.cond = r->cond + (size_t)l * r->H * (r->W + 1);
        d.total = r->total + l;
      }
    }
    NPG_HIP_CHECK(sl.ctx, hipMemcpyAsync(sl.desc_dev, sl.desc_host, L * sizeof(npg_leaf_desc),
                                         hipMemcpyHostToDevice, sl.stream));
    int rc = npg_run_desc_batch(sl.ctx, model, precision, sl.desc_dev, L, batch[0]->H, batch[0]->W, sl.stream);
    if (rc) return rc;
    for (const Req *r : batch) {  // each request owns an event recorded at the same point
      hipEvent_t e = nullptr;
      NPG_HIP_CHECK(sl.ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      NPG_HIP_CHECK(sl.ctx, hipEventRecord(e, sl.stream));
      ready[r->id] = e;
    }
    NPG_HIP_CHECK(sl.ctx, hipEventRecord(sl.done, sl.stream));
    return NPG_OK;
  }
};

}  // namespace

struct npg_server {
  npg_ctx *parent = nullptr;
  const npg_model *model = nullptr;
  npg_serve_params prm{};
  void *arena_dev = nullptr;
  HipExec ex;
  npg_serve_core::Core<HipExec> core;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stop = false;

  void loop();
};

void npg_server::loop() {
  (void)hipSetDevice(parent->device);
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    const bool done = core.completions();
    core.admit();
    if (done) cv_done.notify_all();
    if (core.busy())
      cv_work.wait_for(lk, std::chrono::microseconds(20));
    else
      cv_work.wait_for(lk, std::chrono::milliseconds(2));
  }
}

extern "C" {

int npg_serve_create(npg_ctx *ctx, const npg_model *model, const npg_serve_params *prm, npg_server **out) {
  if (!ctx || !model || !prm || !out) return NPG_E_ARG;
  *out = nullptr;
  if (prm->n_slots < 1 || prm->n_slots > 16 || prm->table_bytes == 0)
    return npg_fail(ctx, NPG_E_ARG, "serve: n_slots in [1,16] and table_bytes > 0 required");
  if (prm->precision != NPG_FP32 && prm->precision != NPG_BF16 && prm->precision != NPG_FP8)
    return npg_fail(ctx, NPG_E_ARG, "serve: bad precision %d", (int)prm->precision);
  if (prm->precision == NPG_FP8 && !npg_model_fp8_ready(model))
    return npg_fail(ctx, NPG_E_ARG, "serve: FP8 needs npg_model_calibrate_fp8 first");
  if (npg_model_in_channels(model) != 1)
    return npg_fail(ctx, NPG_E_ARG, "serve: one-channel models only");
  int rc = npg_set_device(ctx);
  if (rc) return rc;
  npg_server *sv = new npg_server();
  sv->parent = ctx;
  sv->model = model;
  sv->prm = *prm;
  rc = npg_device_alloc(ctx, prm->table_bytes, &sv->arena_dev);
  if (rc) {
    delete sv;
    return rc;
  }
  sv->ex.model = model;
  sv->ex.precision = prm->precision;
  sv->ex.slots.resize(prm->n_slots);
  sv->core.init(&sv->ex, (int)prm->n_slots, prm->max_batch_leaves, sv->arena_dev, prm->table_bytes);
  for (Slot &sl : sv->ex.slots) {
    rc = npg_create(&sl.ctx, ctx->device, prm->slot_scratch_bytes);
    if (!rc && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) rc = NPG_E_HIP;
    if (!rc && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) rc = NPG_E_HIP;
    if (rc) break;
  }
  if (rc) {
    npg_serve_destroy(sv);
    return npg_fail(ctx, rc, "serve: slot creation failed");
  }
  sv->th = std::thread([sv] { sv->loop(); });
  *out = sv;
  return NPG_OK;
}

void npg_serve_destroy(npg_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->th.joinable()) sv->th.join();
  (void)hipSetDevice(sv->parent->device);
  for (Slot &sl : sv->ex.slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  }
  for (auto &kv : sv->ex.ready) (void)hipEventDestroy(kv.second);
  sv->ex.ready.clear();
  for (Slot &sl : sv->ex.slots) {
    if (sl.desc_dev) (void)hipFree(sl.desc_dev);
    if (sl.desc_host) (void)hipHostFree(sl.desc_host);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ctx) npg_destroy(sl.ctx);
  }
  npg_device_free(sv->parent, sv->arena_dev, sv->prm.table_bytes);
  delete sv;
}

int npg_serve_submit_recon(npg_server *sv, const float *dir_dev, const uint32_t *w_dev,
                           const uint32_t *leaf_begin_host, const uint32_t *leaf_count_host, uint32_t L, int H, int W,
                           uint64_t *ticket) {
  if (!sv || !ticket) return NPG_E_ARG;
  if (!pow2_in(H, 4, 1024) || !pow2_in(W, 4, 1024) || L == 0 || !dir_dev || !w_dev || !leaf_begin_host ||
      !leaf_count_host)
    return npg_fail(sv->parent, NPG_E_ARG, "serve: bad reconstruction request");
  if (!npg_model_fits(sv->model, H, W))
    return npg_fail(sv->parent, NPG_E_ARG, "serve: the network's levels do not divide %dx%d", H, W);
  Req r;
  r.dir = dir_dev;
  r.w = w_dev;
  r.beg.assign(leaf_begin_host, leaf_begin_host + L);
  r.cnt.assign(leaf_count_host, leaf_count_host + L);
  r.L = L;
  r.H = H;
  r.W = W;
  int rc;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    rc = sv->core.submit_recon(std::move(r), ticket);
    if (rc) npg_fail(sv->parent, rc, "%s", sv->core.error.c_str());
  }
  if (!rc) sv->cv_work.notify_all();
  return rc;
}

int npg_serve_submit_sample(npg_server *sv, uint64_t recon_ticket, const uint32_t *leaf_dev, const float *u_dev,
                            uint64_t n, float *dir_out_dev, float *pdf_out_dev, uint64_t *ticket) {
  if (!sv || !ticket || !leaf_dev || !u_dev || !dir_out_dev || !pdf_out_dev || n == 0)
    return NPG_E_ARG;
  Req r;
  r.recon = recon_ticket;
  r.leaf = leaf_dev;
  r.u = u_dev;
  r.n = n;
  r.dir_out = dir_out_dev;
  r.pdf_out = pdf_out_dev;
  int rc;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    rc = sv->core.submit_sample(std::move(r), ticket);
    if (rc) npg_fail(sv->parent, rc, "%s", sv->core.error.c_str());
  }
  if (!rc) sv->cv_work.notify_all();
  return rc;
}

int npg_serve_poll(npg_server *sv, uint64_t ticket, double *latency_us) {
  if (!sv) return NPG_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  return sv->core.poll(ticket, latency_us);
}

int npg_serve_wait(npg_server *sv, uint64_t ticket, double *latency_us) {
  if (!sv) return NPG_E_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    const int r = sv->core.poll(ticket, latency_us);
    if (r != 0) return r;
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(5));
  }
}

int npg_serve_tables(npg_server *sv, uint64_t ticket, npg_tables *out) {
  if (!sv || !out) return NPG_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  return sv->core.tables(ticket, out);
}

const char *npg_serve_last_error(npg_server *sv) {
  thread_local std::string copy;
  if (!sv) return "";
  std::lock_guard<std::mutex> lk(sv->mu);
  copy = sv->core.error;
  return copy.c_str();
}

int npg_serve_release(npg_server *sv, uint64_t ticket) {
  if (!sv) return NPG_E_ARG;
  int rc;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    rc = sv->core.release(ticket);
  }
  sv->cv_work.notify_all();
  return rc;
}

int npg_serve_copy_tables(npg_server *sv, uint64_t ticket, float *pdf_dev, float *marg_dev, float *cond_dev,
                          double *total_dev, void *stream) {
  npg_tables t;
  int rc = npg_serve_tables(sv, ticket, &t);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t HW = (size_t)t.H * t.W;
  NPG_HIP_CHECK(sv->parent, hipMemcpyAsync(pdf_dev, t.pdf_dev, t.L * HW * 4, hipMemcpyDeviceToDevice, s));
  NPG_HIP_CHECK(sv->parent, hipMemcpyAsync(marg_dev, t.marg_dev, t.L * (size_t)(t.H + 1) * 4, hipMemcpyDeviceToDevice, s));
  NPG_HIP_CHECK(sv->parent,
                hipMemcpyAsync(cond_dev, t.cond_dev, t.L * (size_t)t.H * (t.W + 1) * 4, hipMemcpyDeviceToDevice, s));
  if (total_dev) NPG_HIP_CHECK(sv->parent, hipMemcpyAsync(total_dev, t.total_dev, t.L * 8, hipMemcpyDeviceToDevice, s));
  return NPG_OK;
}

void npg_serve_get_stats(npg_server *sv, npg_serve_stats *out) {
  if (!sv || !out) return;
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->core.get_stats(out);
}

}  // extern "C"
