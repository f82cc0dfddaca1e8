// Scheduling core of the request server (continuous batching of
// reconstruction and sampling requests), free of device calls so that the
// same code runs under the HIP executor of serve.hip and under a fake
// executor in host-only tests.
//
//  - Requests wait in one FIFO.  Whenever a slot is free, admit() takes the
//    oldest launchable request.  A sampling request is launchable once its
//    reconstruction has been launched (it then waits for that batch on the
//    device).  A reconstruction is batched with every later waiting
//    reconstruction of the same map size, up to max_batch_leaves leaves and
//    while their tables fit in the table arena; a reconstruction whose
//    tables do not fit yet blocks later reconstructions (FIFO) but not
//    sampling requests, which need no table memory.
//  - Tables stay in the arena until the client releases the request and no
//    sampling request against them is pending or running.
//  - completions() asks the executor which busy slots have finished and
//    retires their requests.
//
// The executor provides:
//   double now_us();
//   int launch_recon(int slot, const std::vector<Req *> &batch, uint32_t leaves);
//   int launch_sample(int slot, Req &sample, const Req &recon);
//   int query(int slot);            // 0 running, 1 finished, < 0 failed
//   const char *slot_error(int slot);
//   void forget(Req &r);            // drop per-request device state (events)
// Every method of Core is called with the server's lock held.
#pragma once

#include <stdint.h>
#include <stddef.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <string>
#include <vector>

#include "../../include/npg.h"

namespace npg_serve_core {

enum State { QUEUED = 0, RUNNING = 1, DONE = 2, FAILED = 3 };
enum Kind { RECON = 0, SAMPLE = 1 };

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Bytes of one request's tables in the arena: pdf [L][H][W], marg
// [L][H+1], cond [L][H][W+1] (float32), total [L] (binary64), each piece
// 256-byte aligned.
inline size_t table_bytes(uint32_t L, int H, int W) {
  const size_t HW = (size_t)H * W;
  return align256(L * HW * 4) + align256(L * (size_t)(H + 1) * 4) + align256(L * (size_t)H * (W + 1) * 4) +
         align256((size_t)L * 8);
}

struct Req {
  uint64_t id = 0;
  int kind = RECON;
  int state = QUEUED;
  int rc = NPG_OK;
  bool release_on_done = false;
  int users = 0;  // sampling requests submitted against the tables, not yet done
  double t_submit = 0, t_start = 0, t_done = 0;
  // reconstruction
  const float *dir = nullptr;
  const uint32_t *w = nullptr;
  std::vector<uint32_t> beg, cnt;
  uint32_t L = 0;
  int H = 0, W = 0;
  size_t off = 0, bytes = 0;  // table block in the arena (bytes set at submission)
  bool has_block = false;     // the block is held (from admission until freed)
  float *pdf = nullptr, *marg = nullptr, *cond = nullptr;
  double *total = nullptr;
  // sampling
  uint64_t recon = 0;
  const uint32_t *leaf = nullptr;
  const float *u = nullptr;
  uint64_t n = 0;
  float *dir_out = nullptr, *pdf_out = nullptr;
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

struct SlotState {
  bool busy = false;
  std::vector<uint64_t> tickets;
};

template <class Exec>
struct Core {
  Exec *ex = nullptr;
  uint32_t max_batch_leaves = 0;  // 0: no merging
  char *arena_base = nullptr;     // device address of the arena
  Arena arena;
  std::vector<SlotState> slots;
  std::map<uint64_t, Req> reqs;
  std::deque<uint64_t> pending;
  uint64_t next_id = 1;
  npg_serve_stats stats{};
  std::string error;

  void init(Exec *e, int n_slots, uint32_t max_leaves, void *base, size_t table_bytes_total) {
    ex = e;
    max_batch_leaves = max_leaves;
    arena_base = static_cast<char *>(base);
    arena.init(table_bytes_total);
    slots.assign((size_t)n_slots, SlotState{});
  }

  int unknown(uint64_t ticket) {
    error = "serve: unknown or released ticket " + std::to_string(ticket);
    return NPG_E_ARG;
  }

  // A reconstruction request (beg/cnt/L/H/W/dir/w filled in); NPG_E_BUDGET if
  // its tables can never fit in the arena.
  int submit_recon(Req r, uint64_t *ticket) {
    r.kind = RECON;
    r.bytes = table_bytes(r.L, r.H, r.W);
    if (r.bytes > arena.size) {
      error = "serve: tables of " + std::to_string(r.L) + " leaves exceed the table arena";
      return NPG_E_BUDGET;
    }
    r.t_submit = ex->now_us();
    r.id = next_id++;
    *ticket = r.id;
    pending.push_back(r.id);
    reqs.emplace(r.id, std::move(r));
    ++stats.submitted;
    return NPG_OK;
  }

  // A sampling request against the reconstruction r.recon.
  int submit_sample(Req r, uint64_t *ticket) {
    auto it = reqs.find(r.recon);
    if (it == reqs.end() || it->second.kind != RECON) {
      error = "serve: unknown reconstruction ticket";
      return NPG_E_ARG;
    }
    r.kind = SAMPLE;
    ++it->second.users;  // the tables stay until this request is done
    r.t_submit = ex->now_us();
    r.id = next_id++;
    *ticket = r.id;
    pending.push_back(r.id);
    reqs.emplace(r.id, std::move(r));
    ++stats.submitted;
    return NPG_OK;
  }

  // 1 done (latency set), 0 not yet, < 0 failed or unknown.
  int poll(uint64_t ticket, double *latency_us) {
    auto it = reqs.find(ticket);
    if (it == reqs.end()) return unknown(ticket);
    const Req &r = it->second;
    if (r.state == FAILED) return r.rc ? r.rc : NPG_E_HIP;
    if (r.state != DONE) return 0;
    if (latency_us) *latency_us = r.t_done - r.t_submit;
    return 1;
  }

  int tables(uint64_t ticket, npg_tables *out) {
    auto it = reqs.find(ticket);
    if (it == reqs.end()) return unknown(ticket);
    if (it->second.kind != RECON || it->second.state != DONE) {
      error = "serve: tables of a request that is not a finished reconstruction";
      return NPG_E_ARG;
    }
    const Req &r = it->second;
    *out = npg_tables{r.pdf, r.marg, r.cond, r.total, r.L, r.H, r.W};
    return NPG_OK;
  }

  // A queued reconstruction holds no block yet: only admitted ones give
  // theirs back.
  void free_tables(Req &r) {
    if (r.kind == RECON && r.has_block) {
      arena.release(r.off, r.bytes);
      r.has_block = false;
    }
    ex->forget(r);
  }

  // A sampling request against `recon` has finished (or failed, or was
  // released before it ran): the tables go once they are released and unused.
  void drop_user(uint64_t recon) {
    auto rr = reqs.find(recon);
    if (rr == reqs.end()) return;
    Req &rc = rr->second;
    if (--rc.users == 0 && rc.release_on_done && (rc.state == DONE || rc.state == FAILED)) {
      free_tables(rc);
      reqs.erase(rr);
    }
  }

  int release(uint64_t ticket) {
    auto it = reqs.find(ticket);
    if (it == reqs.end()) return unknown(ticket);
    Req &r = it->second;
    if (r.state == RUNNING || r.users > 0) {
      r.release_on_done = true;
      return NPG_OK;
    }
    if (r.state == QUEUED)
      for (auto p = pending.begin(); p != pending.end(); ++p)
        if (*p == ticket) {
          pending.erase(p);
          break;
        }
    const bool queued_sample = r.kind == SAMPLE && r.state == QUEUED;
    const uint64_t recon = r.recon;
    free_tables(r);
    reqs.erase(it);
    if (queued_sample) drop_user(recon);
    return NPG_OK;
  }

  bool busy() const {
    for (const SlotState &s : slots)
      if (s.busy) return true;
    return false;
  }

  bool completions() {
    bool any = false;
    for (size_t si = 0; si < slots.size(); ++si) {
      SlotState &sl = slots[si];
      if (!sl.busy) continue;
      const int q = ex->query((int)si);
      if (q == 0) continue;
      const double t = ex->now_us();
      for (uint64_t id : sl.tickets) {
        auto it = reqs.find(id);
        if (it == reqs.end()) continue;
        Req &r = it->second;
        r.state = q > 0 ? DONE : FAILED;
        if (q < 0) {
          r.rc = NPG_E_HIP;
          error = std::string("serve: batch failed on the device: ") + ex->slot_error((int)si);
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

  void admit() {
    for (size_t si = 0; si < slots.size(); ++si) {
      SlotState &sl = slots[si];
      if (sl.busy) continue;
      bool recon_blocked = false, launched = false;
      std::vector<uint64_t> batch;
      for (auto pit = pending.begin(); pit != pending.end() && !launched; ++pit) {
        Req &head = reqs.at(*pit);
        const double t = ex->now_us();
        if (head.kind == SAMPLE) {
          auto rr = reqs.find(head.recon);
          if (rr != reqs.end() && rr->second.state == QUEUED) continue;
          const uint64_t id = head.id;
          pending.erase(pit);
          head.t_start = t;
          const bool orphan = rr == reqs.end() || rr->second.state == FAILED;
          const int rc = orphan ? NPG_E_ARG : ex->launch_sample((int)si, head, rr->second);
          if (rc) {
            error = orphan ? "serve: sampling request against a failed reconstruction" : ex->slot_error((int)si);
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
        // this request plus later waiting requests of the same map size,
        // while leaves and table memory allow
        uint32_t leaves = 0;
        std::vector<Req *> rs;
        for (auto it = pit; it != pending.end(); ++it) {
          Req &r = reqs.at(*it);
          if (r.kind != RECON || r.H != head.H || r.W != head.W) continue;
          if (!batch.empty() && (max_batch_leaves == 0 || leaves + r.L > max_batch_leaves)) continue;
          size_t off = 0;
          if (!arena.alloc(r.bytes, &off)) break;  // FIFO among reconstructions
          r.off = off;
          r.has_block = true;
          char *base = arena_base + off;
          const size_t HW = (size_t)r.H * r.W;
          const size_t o1 = align256(r.L * HW * 4), o2 = o1 + align256(r.L * (size_t)(r.H + 1) * 4);
          const size_t o3 = o2 + align256(r.L * (size_t)r.H * (r.W + 1) * 4);
          r.pdf = reinterpret_cast<float *>(base);
          r.marg = reinterpret_cast<float *>(base + o1);
          r.cond = reinterpret_cast<float *>(base + o2);
          r.total = reinterpret_cast<double *>(base + o3);
          batch.push_back(r.id);
          rs.push_back(&r);
          leaves += r.L;
          if (max_batch_leaves == 0) break;
        }
        if (batch.empty()) {
          recon_blocked = true;
          continue;
        }
        // by id: erasing inside a deque invalidates every iterator into it
        pending.erase(std::remove_if(pending.begin(), pending.end(),
                                     [&rs](uint64_t id) {
                                       for (const Req *r : rs)
                                         if (r->id == id) return true;
                                       return false;
                                     }),
                      pending.end());
        const int rc = ex->launch_recon((int)si, rs, leaves);
        for (Req *r : rs) {
          r->t_start = t;
          if (rc) {
            r->state = FAILED;
            r->rc = rc;
            r->t_done = t;
            free_tables(*r);
          } else {
            r->state = RUNNING;
          }
        }
        if (rc) {
          error = ex->slot_error((int)si);
          break;
        }
        ++stats.batches;
        stats.leaves += leaves;
        if (batch.size() > 1) stats.merged_requests += batch.size() - 1;
        sl.tickets = batch;
        sl.busy = true;
        launched = true;
        break;
      }
      if (!launched) return;
      uint64_t n_busy = 0;
      for (const SlotState &x : slots) n_busy += x.busy;
      if (n_busy > stats.max_concurrent) stats.max_concurrent = n_busy;
    }
  }

  void get_stats(npg_serve_stats *out) const {
    *out = stats;
    out->queued = pending.size();
    out->table_bytes_free = arena.free_bytes();
  }
};

}  // namespace npg_serve_core
