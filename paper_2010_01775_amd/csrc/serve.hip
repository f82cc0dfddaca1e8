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

int npg_run_desc_batch(npg_ctx *ctx, const npg_model *m, npg_precision prec, const npg_leaf_desc *d_dev,
                       uint32_t L, int H, int W, hipStream_t s);

namespace {

using Clock = std::chrono::steady_clock;

double now_us() {
  return std::chrono::duration<double, std::micro>(Clock::now().time_since_epoch()).count();
}

enum State { QUEUED = 0, RUNNING = 1, DONE = 2, FAILED = 3 };
enum Kind { RECON = 0, SAMPLE = 1 };

struct Req {
  uint64_t id = 0;
  int kind = RECON;
  int state = QUEUED;
  int rc = NPG_OK;
  bool release_on_done = false;
  int users = 0;               // sampling requests submitted against the tables, not yet done
  double t_submit = 0, t_start = 0, t_done = 0;
  // reconstruction
  const float *dir = nullptr;
  const uint32_t *w = nullptr;
  std::vector<uint32_t> beg, cnt;
  uint32_t L = 0;
  int H = 0, W = 0;
  size_t off = 0, bytes = 0;  // table block in the arena
  float *pdf = nullptr, *marg = nullptr, *cond = nullptr;
  double *total = nullptr;
  hipEvent_t ready = nullptr;  // recorded after the batch that computed the tables
  // sampling
  uint64_t recon = 0;
  const uint32_t *leaf = nullptr;
  const float *u = nullptr;
  uint64_t n = 0;
  float *dir_out = nullptr, *pdf_out = nullptr;
};

struct Slot {
  npg_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
  npg_leaf_desc *desc_dev = nullptr;
  npg_leaf_desc *desc_host = nullptr;  // pinned
  size_t desc_cap = 0;
};

// Best-fit allocator over [0, size) with coalescing of free ranges.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(size_t n) {
    size = n;
    free_.clear();
    if (n) free_[0] = n;
  }
  bool alloc(size_t n, size_t *off) {
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n && (best == free_.end() || it->second < best->second)) best = it;
    if (best == free_.end()) return false;
    *off = best->first;
    const size_t rest = best->second - n;
    const size_t at = best->first + n;
    free_.erase(best);
    if (rest) free_[at] = rest;
    return true;
  }
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t s = 0;
    for (auto &kv : free_) s += kv.second;
    return s;
  }
};

size_t table_bytes(uint32_t L, int H, int W) {
  const size_t HW = (size_t)H * W;
  return npg_align(L * HW * 4) + npg_align(L * (size_t)(H + 1) * 4) + npg_align(L * (size_t)H * (W + 1) * 4) +
         npg_align(L * 8);
}

}  // namespace

struct npg_server {
  npg_ctx *parent = nullptr;
  const npg_model *model = nullptr;
  npg_serve_params prm{};
  std::vector<Slot> slots;
  void *arena_dev = nullptr;
  Arena arena;
  std::map<uint64_t, Req> reqs;
  std::deque<uint64_t> pending;
  uint64_t next_id = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stop = false;
  npg_serve_stats stats{};
  std::string error;

  void loop();
  bool completions();
  void admit();
  int launch_recon(Slot &sl, std::vector<uint64_t> &batch);
  int run_sample(Slot &sl, Req &r);
  void free_tables(Req &r);
  void drop_user(uint64_t recon);
  int unknown(uint64_t ticket) {
    error = "serve: unknown or released ticket " + std::to_string(ticket);
    return NPG_E_ARG;
  }
};

void npg_server::free_tables(Req &r) {
  if (r.kind == RECON && r.bytes) {
    arena.release(r.off, r.bytes);
    r.bytes = 0;
  }
  if (r.ready) {
    (void)hipEventDestroy(r.ready);
    r.ready = nullptr;
  }
}

// A sampling request against `recon` has finished (or failed, or was
// released before it ran): the tables go once they are released and unused.
void npg_server::drop_user(uint64_t recon) {
  auto rr = reqs.find(recon);
  if (rr == reqs.end()) return;
  Req &rc = rr->second;
  if (--rc.users == 0 && rc.release_on_done && (rc.state == DONE || rc.state == FAILED)) {
    free_tables(rc);
    reqs.erase(rr);
  }
}

bool npg_server::completions() {
  bool any = false;
  for (Slot &sl : slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    const double t = now_us();
    for (uint64_t id : sl.tickets) {
      auto it = reqs.find(id);
      if (it == reqs.end()) continue;
      Req &r = it->second;
      r.state = q == hipSuccess ? DONE : FAILED;
      if (q != hipSuccess) {
        r.rc = NPG_E_HIP;
        error = std::string("serve: batch failed on the device: ") + hipGetErrorString(q);
      }
      r.t_done = t;
      ++stats.completed;
      if (r.kind == SAMPLE) {
        drop_user(r.recon);
        it = reqs.find(id);
      }
      if (it != reqs.end() && it->second.release_on_done && it->second.users == 0) {
        free_tables(it->second);
        reqs.erase(it);
      }
    }
    sl.tickets.clear();
    sl.busy = false;
    any = true;
  }
  return any;
}

int npg_server::run_sample(Slot &sl, Req &r) {
  Req &rc = reqs.at(r.recon);
  if (rc.ready) NPG_HIP_CHECK(sl.ctx, hipStreamWaitEvent(sl.stream, rc.ready, 0));
  npg_tables t{rc.pdf, rc.marg, rc.cond, rc.total, rc.L, rc.H, rc.W};
  NPG_HIP_CHECK(sl.ctx, launch_sample(t, r.leaf, r.u, r.n, r.dir_out, r.pdf_out, nullptr, sl.ctx->err_dev, sl.stream));
  NPG_HIP_CHECK(sl.ctx, hipEventRecord(sl.done, sl.stream));
  return NPG_OK;
}

int npg_server::launch_recon(Slot &sl, std::vector<uint64_t> &batch) {
  uint32_t L = 0;
  for (uint64_t id : batch) L += reqs.at(id).L;
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
  const Req &r0 = reqs.at(batch[0]);
  for (uint64_t id : batch) {
    const Req &r = reqs.at(id);
    const size_t HW = (size_t)r.H * r.W;
    for (uint32_t l = 0; l < r.L; ++l, ++k) {
      npg_leaf_desc &d = sl.desc_host[k];
      d.dir = r.dir;
      d.w = r.w;
      d.begin = r.beg[l];
      d.count = r.cnt[l];
      d.pdf = r.pdf + l * HW;
      d.marg = r.marg + (size_t)l * (r.H + 1);
      d.cond = r.cond + (size_t)l * r.H * (r.W + 1);
      d.total = r.total + l;
    }
  }
  NPG_HIP_CHECK(sl.ctx, hipMemcpyAsync(sl.desc_dev, sl.desc_host, L * sizeof(npg_leaf_desc), hipMemcpyHostToDevice,
                                       sl.stream));
  int rc = npg_run_desc_batch(sl.ctx, model, prm.precision, sl.desc_dev, L, r0.H, r0.W, sl.stream);
  if (rc) return rc;
  hipEvent_t ev = nullptr;
  NPG_HIP_CHECK(sl.ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  NPG_HIP_CHECK(sl.ctx, hipEventRecord(ev, sl.stream));
  for (size_t i = 0; i < batch.size(); ++i) {
    Req &r = reqs.at(batch[i]);
    if (i == 0) {
      r.ready = ev;
    } else {
      // each request owns an event recorded at the same point
      hipEvent_t e2 = nullptr;
      NPG_HIP_CHECK(sl.ctx, hipEventCreateWithFlags(&e2, hipEventDisableTiming));
      NPG_HIP_CHECK(sl.ctx, hipEventRecord(e2, sl.stream));
      r.ready = e2;
    }
  }
  NPG_HIP_CHECK(sl.ctx, hipEventRecord(sl.done, sl.stream));
  ++stats.batches;
  stats.leaves += L;
  if (batch.size() > 1) stats.merged_requests += batch.size() - 1;
  return NPG_OK;
}

void npg_server::admit() {
  for (Slot &sl : slots) {
    if (sl.busy) continue;
    // First launchable request in FIFO order.  A sampling request waits
    // until its reconstruction has been launched; a reconstruction whose
    // tables do not fit yet blocks later reconstructions (FIFO) but not
    // sampling requests, which need no table memory.
    bool recon_blocked = false, launched = false;
    std::vector<uint64_t> batch;
    for (auto pit = pending.begin(); pit != pending.end() && !launched; ++pit) {
      Req &head = reqs.at(*pit);
      const double t = now_us();
      if (head.kind == SAMPLE) {
        auto rr = reqs.find(head.recon);
        if (rr != reqs.end() && rr->second.state == QUEUED) continue;
        const uint64_t id = head.id;
        pending.erase(pit);
        head.t_start = t;
        const bool orphan = rr == reqs.end() || rr->second.state == FAILED;
        const int rc = orphan ? NPG_E_ARG : run_sample(sl, head);
        if (rc) {
          error = orphan ? "serve: sampling request against a failed reconstruction" : sl.ctx->last_error;
          head.state = FAILED;
          head.rc = rc;
          head.t_done = t;
          drop_user(head.recon);
          break;  // iterator invalidated; the next round retries
        }
        head.state = RUNNING;
        sl.tickets = {id};
        sl.busy = true;
        launched = true;
        break;
      }
      if (recon_blocked) continue;
      // reconstruction batch: this request plus later waiting requests of
      // the same map size, while leaves and table memory allow
      uint32_t leaves = 0;
      std::vector<std::deque<uint64_t>::iterator> take;
      for (auto it = pit; it != pending.end(); ++it) {
        Req &r = reqs.at(*it);
        if (r.kind != RECON || r.H != head.H || r.W != head.W) continue;
        if (!batch.empty() && (prm.max_batch_leaves == 0 || leaves + r.L > prm.max_batch_leaves)) continue;
        size_t off = 0;
        if (!arena.alloc(r.bytes, &off)) break;  // FIFO among reconstructions
        r.off = off;
        char *base = static_cast<char *>(arena_dev) + off;
        const size_t HW = (size_t)r.H * r.W;
        const size_t o1 = npg_align(r.L * HW * 4), o2 = o1 + npg_align(r.L * (size_t)(r.H + 1) * 4);
        const size_t o3 = o2 + npg_align(r.L * (size_t)r.H * (r.W + 1) * 4);
        r.pdf = reinterpret_cast<float *>(base);
        r.marg = reinterpret_cast<float *>(base + o1);
        r.cond = reinterpret_cast<float *>(base + o2);
        r.total = reinterpret_cast<double *>(base + o3);
        batch.push_back(r.id);
        take.push_back(it);
        leaves += r.L;
        if (prm.max_batch_leaves == 0) break;
      }
      if (batch.empty()) {
        recon_blocked = true;
        continue;
      }
      for (auto it = take.rbegin(); it != take.rend(); ++it) pending.erase(*it);
      const int rc = launch_recon(sl, batch);
      for (uint64_t id : batch) {
        Req &r = reqs.at(id);
        r.t_start = t;
        if (rc) {
          r.state = FAILED;
          r.rc = rc;
          r.t_done = t;
          free_tables(r);
        } else {
          r.state = RUNNING;
        }
      }
      if (rc) {
        error = sl.ctx->last_error;
        break;
      }
      sl.tickets = batch;
      sl.busy = true;
      launched = true;
      break;
    }
    if (!launched) return;
    int busy = 0;
    for (Slot &x : slots) busy += x.busy;
    if ((uint64_t)busy > stats.max_concurrent) stats.max_concurrent = busy;
  }
}

void npg_server::loop() {
  (void)hipSetDevice(parent->device);
  std::unique_lock<std::mutex> lk(mu);
  while (!stop) {
    const bool done = completions();
    admit();
    if (done) cv_done.notify_all();
    bool busy = false;
    for (Slot &sl : slots) busy |= sl.busy;
    if (busy)
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
  sv->arena.init(prm->table_bytes);
  sv->slots.resize(prm->n_slots);
  for (Slot &sl : sv->slots) {
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
  for (Slot &sl : sv->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  }
  for (auto &kv : sv->reqs)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  for (Slot &sl : sv->slots) {
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
  r.kind = RECON;
  r.dir = dir_dev;
  r.w = w_dev;
  r.beg.assign(leaf_begin_host, leaf_begin_host + L);
  r.cnt.assign(leaf_count_host, leaf_count_host + L);
  r.L = L;
  r.H = H;
  r.W = W;
  r.bytes = table_bytes(L, H, W);
  if (r.bytes > sv->arena.size)
    return npg_fail(sv->parent, NPG_E_BUDGET, "serve: tables of %u leaves exceed the table arena", L);
  r.t_submit = now_us();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    r.id = sv->next_id++;
    *ticket = r.id;
    sv->pending.push_back(r.id);
    sv->reqs.emplace(r.id, std::move(r));
    ++sv->stats.submitted;
  }
  sv->cv_work.notify_all();
  return NPG_OK;
}

int npg_serve_submit_sample(npg_server *sv, uint64_t recon_ticket, const uint32_t *leaf_dev, const float *u_dev,
                            uint64_t n, float *dir_out_dev, float *pdf_out_dev, uint64_t *ticket) {
  if (!sv || !ticket || !leaf_dev || !u_dev || !dir_out_dev || !pdf_out_dev || n == 0)
    return NPG_E_ARG;
  Req r;
  r.kind = SAMPLE;
  r.recon = recon_ticket;
  r.leaf = leaf_dev;
  r.u = u_dev;
  r.n = n;
  r.dir_out = dir_out_dev;
  r.pdf_out = pdf_out_dev;
  r.t_submit = now_us();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(recon_ticket);
    if (it == sv->reqs.end() || it->second.kind != RECON)
      return npg_fail(sv->parent, NPG_E_ARG, "serve: unknown reconstruction ticket");
    ++it->second.users;  // the tables stay until this request is done
    r.id = sv->next_id++;
    *ticket = r.id;
    sv->pending.push_back(r.id);
    sv->reqs.emplace(r.id, std::move(r));
    ++sv->stats.submitted;
  }
  sv->cv_work.notify_all();
  return NPG_OK;
}

int npg_serve_poll(npg_server *sv, uint64_t ticket, double *latency_us) {
  if (!sv) return NPG_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return sv->unknown(ticket);
  const Req &r = it->second;
  if (r.state == FAILED) return r.rc ? r.rc : NPG_E_HIP;
  if (r.state != DONE) return 0;
  if (latency_us) *latency_us = r.t_done - r.t_submit;
  return 1;
}

int npg_serve_wait(npg_server *sv, uint64_t ticket, double *latency_us) {
  if (!sv) return NPG_E_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return sv->unknown(ticket);
    const Req &r = it->second;
    if (r.state == FAILED) return r.rc ? r.rc : NPG_E_HIP;
    if (r.state == DONE) {
      if (latency_us) *latency_us = r.t_done - r.t_submit;
      return 1;
    }
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(5));
  }
}

int npg_serve_tables(npg_server *sv, uint64_t ticket, npg_tables *out) {
  if (!sv || !out) return NPG_E_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return sv->unknown(ticket);
  if (it->second.kind != RECON || it->second.state != DONE) {
    sv->error = "serve: tables of a request that is not a finished reconstruction";
    return NPG_E_ARG;
  }
  const Req &r = it->second;
  *out = npg_tables{r.pdf, r.marg, r.cond, r.total, r.L, r.H, r.W};
  return NPG_OK;
}

const char *npg_serve_last_error(npg_server *sv) {
  thread_local std::string copy;
  if (!sv) return "";
  std::lock_guard<std::mutex> lk(sv->mu);
  copy = sv->error;
  return copy.c_str();
}

int npg_serve_release(npg_server *sv, uint64_t ticket) {
  if (!sv) return NPG_E_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return sv->unknown(ticket);
    Req &r = it->second;
    if (r.state == RUNNING || r.users > 0) {
      r.release_on_done = true;
    } else {
      if (r.state == QUEUED)
        for (auto p = sv->pending.begin(); p != sv->pending.end(); ++p)
          if (*p == ticket) {
            sv->pending.erase(p);
            break;
          }
      const bool queued_sample = r.kind == SAMPLE && r.state == QUEUED;
      const uint64_t recon = r.recon;
      sv->free_tables(r);
      sv->reqs.erase(it);
      if (queued_sample) sv->drop_user(recon);
    }
  }
  sv->cv_work.notify_all();
  return NPG_OK;
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
  *out = sv->stats;
  out->queued = sv->pending.size();
  out->table_bytes_free = sv->arena.free_bytes();
}

}  // extern "C"
