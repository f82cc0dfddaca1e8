// Host-only checks of the request server's scheduling core
// (paper_2010_01775_amd/csrc/serve_core.h) against a fake executor: batch
// merging by map size and leaf cap, FIFO admission under the table budget,
// slot reuse, sampling after its reconstruction, release rules, failures,
// and a randomised run with invariants checked after every step.
// Built and run by tests/test_serve_core.py (with AddressSanitizer and
// UndefinedBehaviorSanitizer); prints "ok" and exits 0 on success.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "serve_core.h"

using npg_serve_core::Core;
using npg_serve_core::Req;
namespace sc = npg_serve_core;

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      exit(1);                                                          \
    }                                                                   \
  } while (0)

struct Launch {
  int slot;
  std::vector<uint64_t> ids;
  bool sample;
};

struct FakeExec {
  double clock = 0;
  std::vector<int> slot_state;      // 0 running, 1 finished, -1 failed
  std::vector<Launch> log;
  std::set<uint64_t> fail_launch;   // reconstruction ids whose batch launch fails
  std::multiset<uint64_t> forgotten;
  std::map<int, std::vector<uint64_t>> running;  // slot -> ids launched there
  double now_us() { return clock += 1.0; }
  const char *slot_error(int) { return "fake failure"; }
  int query(int s) { return slot_state[s]; }
  void forget(Req &r) { forgotten.insert(r.id); }
  int launch_recon(int s, const std::vector<Req *> &batch, uint32_t) {
    Launch l{s, {}, false};
    for (Req *r : batch) {
      l.ids.push_back(r->id);
      if (fail_launch.count(r->id)) return NPG_E_HIP;
    }
    log.push_back(l);
    running[s] = l.ids;
    slot_state[s] = 0;
    return NPG_OK;
  }
  int launch_sample(int s, Req &r, const Req &recon) {
    CHECK(recon.state == sc::RUNNING || recon.state == sc::DONE);  // tables launched before
    log.push_back(Launch{s, {r.id}, true});
    running[s] = {r.id};
    slot_state[s] = 0;
    return NPG_OK;
  }
};

static char g_arena[1];  // the core only does address arithmetic on the base

static Req recon_req(uint32_t L, int H) {
  Req r;
  r.L = L;
  r.H = r.W = H;
  r.beg.assign(L, 0);
  r.cnt.assign(L, 1);
  r.dir = reinterpret_cast<const float *>(16);
  r.w = reinterpret_cast<const uint32_t *>(16);
  return r;
}

static Req sample_req(uint64_t recon) {
  Req r;
  r.recon = recon;
  r.n = 1000;
  return r;
}

static void finish(Core<FakeExec> &c, FakeExec &ex, int slot, int how = 1) {
  ex.slot_state[slot] = how;
  CHECK(c.completions());
}

// Merging, slot reuse, stats.
static void check_merging() {
  FakeExec ex;
  ex.slot_state.assign(2, 1);
  Core<FakeExec> c;
  c.init(&ex, 2, 100, g_arena, 1ull << 40);
  uint64_t a, b, cc, d;
  CHECK(c.submit_recon(recon_req(10, 64), &a) == NPG_OK);
  CHECK(c.submit_recon(recon_req(20, 128), &b) == NPG_OK);
  CHECK(c.submit_recon(recon_req(30, 64), &cc) == NPG_OK);
  CHECK(c.submit_recon(recon_req(70, 64), &d) == NPG_OK);
  c.admit();
  CHECK(ex.log.size() == 2);
  CHECK(ex.log[0].slot == 0 && ex.log[0].ids == std::vector<uint64_t>({a, cc}));  // 10 + 30, 70 would pass 100
  CHECK(ex.log[1].slot == 1 && ex.log[1].ids == std::vector<uint64_t>({b}));
  CHECK(c.stats.batches == 2 && c.stats.merged_requests == 1 && c.stats.max_concurrent == 2);
  CHECK(c.stats.leaves == 60);
  CHECK(c.pending.size() == 1 && c.pending[0] == d);
  c.admit();  // both slots busy: nothing happens
  CHECK(ex.log.size() == 2);
  double lat = -1;
  CHECK(c.poll(a, &lat) == 0);
  finish(c, ex, 0);
  CHECK(c.poll(a, &lat) == 1 && lat > 0 && c.poll(cc, nullptr) == 1 && c.poll(b, nullptr) == 0);
  c.admit();  // slot 0 is reused for d
  CHECK(ex.log.size() == 3 && ex.log[2].slot == 0 && ex.log[2].ids == std::vector<uint64_t>({d}));
  npg_tables t;
  CHECK(c.tables(a, &t) == NPG_OK && t.L == 10 && t.H == 64);
  CHECK(c.tables(b, &t) == NPG_E_ARG);  // still running
  CHECK(c.stats.submitted == 4);
}

// FIFO admission under the table budget; sampling is not blocked by it and
// waits for its reconstruction's launch.
static void check_budget_fifo() {
  FakeExec ex;
  ex.slot_state.assign(3, 1);
  Core<FakeExec> c;
  const size_t one = sc::table_bytes(30, 64, 64);
  c.init(&ex, 3, 4096, g_arena, one + one / 2);
  uint64_t big;
  CHECK(c.submit_recon(recon_req(400, 64), &big) == NPG_E_BUDGET);  // can never fit
  uint64_t r1, r2, r3, s2;
  CHECK(c.submit_recon(recon_req(30, 64), &r1) == NPG_OK);
  CHECK(c.submit_recon(recon_req(30, 64), &r2) == NPG_OK);
  CHECK(c.submit_sample(sample_req(r2), &s2) == NPG_OK);
  CHECK(c.submit_recon(recon_req(1, 64), &r3) == NPG_OK);  // would fit, but FIFO keeps it behind r2
  c.admit();
  CHECK(ex.log.size() == 1 && ex.log[0].ids == std::vector<uint64_t>({r1}));  // r2 does not fit with r1
  CHECK(c.reqs.at(r2).state == sc::QUEUED && c.reqs.at(r3).state == sc::QUEUED);
  CHECK(c.reqs.at(s2).state == sc::QUEUED);  // its reconstruction has not been launched
  finish(c, ex, 0);
  c.admit();
  CHECK(ex.log.size() == 1);  // r1's tables are still held
  CHECK(c.release(r1) == NPG_OK);
  CHECK(c.arena.free_bytes() == c.arena.size);
  c.admit();
  // r2 and r3 merge (same size), then s2 goes to the next free slot
  CHECK(ex.log.size() == 3);
  CHECK(ex.log[1].ids == std::vector<uint64_t>({r2, r3}) && !ex.log[1].sample);
  CHECK(ex.log[2].ids == std::vector<uint64_t>({s2}) && ex.log[2].sample && ex.log[2].slot != ex.log[1].slot);
  CHECK(c.reqs.at(r2).users == 1);
  CHECK(c.release(r2) == NPG_OK);  // running and in use: released when done
  CHECK(c.reqs.count(r2) == 1 && c.reqs.at(r2).release_on_done);
  finish(c, ex, ex.log[1].slot);
  CHECK(c.reqs.count(r2) == 1);  // s2 still uses the tables
  finish(c, ex, ex.log[2].slot);
  CHECK(c.reqs.count(r2) == 0 && c.poll(r2, nullptr) == NPG_E_ARG);  // gone, unknown ticket
  CHECK(c.poll(s2, nullptr) == 1);
  CHECK(c.release(s2) == NPG_OK && c.release(r3) == NPG_OK);
  CHECK(c.arena.free_bytes() == c.arena.size && c.reqs.empty());
}

// A failed batch launch and a failed batch on the device.
static void check_failures() {
  FakeExec ex;
  ex.slot_state.assign(1, 1);
  Core<FakeExec> c;
  c.init(&ex, 1, 4096, g_arena, 1ull << 40);
  uint64_t r1, s1, r2, s2;
  CHECK(c.submit_recon(recon_req(5, 32), &r1) == NPG_OK);
  CHECK(c.submit_sample(sample_req(r1), &s1) == NPG_OK);
  ex.fail_launch.insert(r1);
  c.admit();
  CHECK(c.poll(r1, nullptr) == NPG_E_HIP && !c.busy());
  CHECK(c.arena.free_bytes() == c.arena.size);  // its tables were returned
  c.admit();  // the sampling request against a failed reconstruction fails
  CHECK(c.poll(s1, nullptr) == NPG_E_ARG);
  CHECK(c.submit_recon(recon_req(5, 32), &r2) == NPG_OK);
  CHECK(c.submit_sample(sample_req(r2), &s2) == NPG_OK);
  c.admit();
  finish(c, ex, 0, -1);  // the batch fails on the device
  CHECK(c.poll(r2, nullptr) == NPG_E_HIP && c.error.find("fake failure") != std::string::npos);
  c.admit();
  CHECK(c.poll(s2, nullptr) == NPG_E_ARG);
  for (uint64_t t : {r1, s1, r2, s2}) CHECK(c.release(t) == NPG_OK);
  CHECK(c.reqs.empty() && c.pending.empty() && c.arena.free_bytes() == c.arena.size);
  CHECK(c.release(r1) == NPG_E_ARG);  // already released
}

// Random submissions, releases and completions; invariants after each step.
static void check_random(unsigned seed) {
  std::mt19937 rng(seed);
  FakeExec ex;
  const int slots = 1 + (int)(rng() % 4);
  ex.slot_state.assign(slots, 1);
  Core<FakeExec> c;
  const size_t budget = sc::table_bytes(300, 64, 64);
  c.init(&ex, slots, 1 + rng() % 400, g_arena, budget);
  std::vector<uint64_t> live_recon, live;
  std::map<uint64_t, int> launches;
  size_t seen = 0;
  for (int step = 0; step < 2000; ++step) {
    const unsigned op = rng() % 10;
    uint64_t t;
    if (op < 3) {
      const int H = (rng() % 2) ? 64 : 32;
      if (c.submit_recon(recon_req(1 + rng() % 200, H), &t) == NPG_OK) {
        live_recon.push_back(t);
        live.push_back(t);
      }
    } else if (op < 5 && !live_recon.empty()) {
      const uint64_t r = live_recon[rng() % live_recon.size()];
      if (c.submit_sample(sample_req(r), &t) == NPG_OK) live.push_back(t);
    } else if (op < 7 && !live.empty()) {
      const size_t k = rng() % live.size();
      const uint64_t id = live[k];
      CHECK(c.release(id) == NPG_OK);
      live.erase(live.begin() + k);
      live_recon.erase(std::remove(live_recon.begin(), live_recon.end(), id), live_recon.end());
    } else {
      for (int s = 0; s < slots; ++s)
        if (c.slots[s].busy && rng() % 2) ex.slot_state[s] = (rng() % 50) ? 1 : -1;
      c.completions();
    }
    c.admit();
    for (; seen < ex.log.size(); ++seen)
      for (uint64_t id : ex.log[seen].ids) ++launches[id];
    // invariants: every request launched at most once; busy slots hold
    // running requests; queued requests are pending; held table bytes
    // (requests still owning a block) + free bytes = the arena
    size_t held = 0;
    std::set<uint64_t> pend(c.pending.begin(), c.pending.end());
    CHECK(pend.size() == c.pending.size());
    for (auto &kv : c.reqs) {
      const Req &r = kv.second;
      CHECK(launches[kv.first] <= 1);
      CHECK((r.state == sc::QUEUED) == (pend.count(kv.first) == 1));
      if (r.kind == sc::RECON && r.has_block) held += r.bytes;
      CHECK(!r.has_block || r.state != sc::QUEUED);
      CHECK(r.users >= 0);
    }
    CHECK(held + c.arena.free_bytes() == c.arena.size);
    for (int s = 0; s < slots; ++s)
      for (uint64_t id : c.slots[s].tickets) CHECK(c.reqs.count(id) == 0 || c.reqs.at(id).state == sc::RUNNING);
  }
  // drain: finish everything; where waiting reconstructions need table
  // memory that finished requests still hold, release the oldest of those
  for (int round = 0; round < 100000 && (c.busy() || !c.pending.empty()); ++round) {
    for (int s = 0; s < slots; ++s) ex.slot_state[s] = 1;
    c.completions();
    c.admit();
    if (!c.busy() && !c.pending.empty()) {
      auto k = std::find_if(live.begin(), live.end(), [&](uint64_t id) {
        return c.reqs.count(id) && c.reqs.at(id).state != sc::QUEUED;
      });
      CHECK(k != live.end());  // otherwise nothing could ever free memory: a deadlock
      CHECK(c.release(*k) == NPG_OK);
      live_recon.erase(std::remove(live_recon.begin(), live_recon.end(), *k), live_recon.end());
      live.erase(k);
    }
  }
  CHECK(!c.busy() && c.pending.empty());
  for (uint64_t id : live) CHECK(c.release(id) == NPG_OK);
  CHECK(c.reqs.empty());
  CHECK(c.arena.free_bytes() == c.arena.size);
}

// Releasing a reconstruction that is still queued gives back no table
// memory (it holds none yet); the arena stays consistent.
static void check_release_queued() {
  FakeExec ex;
  ex.slot_state.assign(1, 1);
  Core<FakeExec> c;
  const size_t one = sc::table_bytes(10, 32, 32);
  c.init(&ex, 1, 4096, g_arena, 2 * one);
  uint64_t r1, r2, r3;
  CHECK(c.submit_recon(recon_req(10, 32), &r1) == NPG_OK);
  c.admit();  // r1 holds one block and its slot
  CHECK(c.submit_recon(recon_req(10, 32), &r2) == NPG_OK);
  CHECK(c.release(r2) == NPG_OK);  // queued: nothing to give back
  CHECK(c.arena.free_bytes() == one);
  CHECK(c.submit_recon(recon_req(10, 32), &r3) == NPG_OK);
  finish(c, ex, 0);
  c.admit();
  CHECK(c.reqs.at(r3).state == sc::RUNNING && c.arena.free_bytes() == 0);
  finish(c, ex, 0);
  CHECK(c.release(r1) == NPG_OK && c.release(r3) == NPG_OK);
  CHECK(c.arena.free_bytes() == c.arena.size && c.arena.free_.size() == 1);
}

int main() {
  check_release_queued();
  check_merging();
  check_budget_fifo();
  check_failures();
  for (unsigned s = 1; s <= 8; ++s) check_random(s);
  printf("ok\n");
  return 0;
}
