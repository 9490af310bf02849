// CPU test of the server's scheduling core with a fake executor: budget
// invariant, strict FIFO admission, refusal of oversize requests, the
// watchdog, and the arena allocator.  Built with g++ (optionally under
// AddressSanitizer/UBSan) by tests/test_sched_native.py.
#include <cassert>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "../../paper_2310_17864_amd/csrc/sched.hpp"

using namespace ctca;

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "CHECK failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

// Completes request k of a launch after lag + ticket % 3 polls (requests of
// one launch finish at different times); a request with `user` set never
// completes, nor does its launch, and one listed in stuck_once hangs in its
// first launch only.  Tracks the charge on the "device".
struct FakeExec {
  struct Handle {
    int polls = 0;
    std::vector<char> stuck, fin;
  };
  int lag = 3;
  int cap = 64;
  int launches_open = 0;
  size_t device_charge = 0, peak = 0, budget = 0;
  bool violated = false;
  std::vector<uint64_t> admit_order;
  std::set<uint64_t> not_ready;     // tickets whose inputs are not written yet
  std::set<uint64_t> stuck_once;    // tickets that hang in their first launch
  int timeouts_seen = 0;
  void on_timeout(Handle&) { ++timeouts_seen; }
  bool ready(const SchedReq* r) const { return not_ready.count(r->ticket) == 0; }
  bool can_launch() const { return launches_open < 8; }
  int max_batch() const { return cap; }
  Handle launch(std::vector<SchedReq*>& reqs) {
    Handle h;
    for (auto* r : reqs) {
      admit_order.push_back(r->ticket);
      device_charge += r->charge;
      h.stuck.push_back(r->user != nullptr || (stuck_once.count(r->ticket) && r->retries == 0));
      h.fin.push_back(0);
    }
    peak = std::max(peak, device_charge);
    if (device_charge > budget) violated = true;
    ++launches_open;
    return h;
  }
  bool poll(Handle& h, const std::vector<SchedReq*>& reqs, std::vector<int>& st) {
    ++h.polls;
    st.assign(reqs.size(), -1);
    bool all = true;
    for (size_t k = 0; k < reqs.size(); ++k) {
      if (!h.stuck[k] && h.polls >= lag + (int)(reqs[k]->ticket % 3)) {
        if (!h.fin[k]) device_charge -= reqs[k]->charge;
        h.fin[k] = 1;
        st[k] = 0;
      } else {
        all = false;
      }
    }
    return all;
  }
  void release(Handle&) { --launches_open; }
};

static void test_budget_fifo() {
  std::mt19937_64 rng(7);
  const size_t budget = 1000;
  FakeExec ex;
  ex.budget = budget;
  Scheduler<FakeExec> s(&ex, budget, 4096, 1 << 20, 0.0);
  std::vector<SchedReq> reqs(2000);
  size_t next = 0, done = 0;
  uint64_t t = 1;
  while (done < reqs.size()) {
    // a random number of arrivals per round
    const int arrivals = (int)(rng() % 4);
    for (int a = 0; a < arrivals && next < reqs.size(); ++a) {
      SchedReq& r = reqs[next++];
      r.ticket = t++;
      r.charge = 1 + rng() % 400;
      r.ws_bytes = 256 * (1 + rng() % 3);
      CHECK(s.submit(&r, 1 << 20) == 0);
    }
    auto fin = s.step();
    done += fin.size();
    CHECK(s.charge_inflight() <= budget);
  }
  CHECK(!ex.violated);
  CHECK(ex.peak <= budget);
  CHECK(!s.stats().budget_violated);
  // strict FIFO: admitted in submission order
  for (size_t i = 1; i < ex.admit_order.size(); ++i) CHECK(ex.admit_order[i] > ex.admit_order[i - 1]);
  CHECK(ex.admit_order.size() == reqs.size());
  CHECK(s.idle());
  CHECK(s.arena().used() == 0);
}

static void test_refusals() {
  FakeExec ex;
  ex.budget = 100;
  Scheduler<FakeExec> s(&ex, 100, 1024, 10, 0.0);
  SchedReq big;
  big.charge = 101;
  big.ws_bytes = 256;
  CHECK(s.submit(&big, 16) == 3);            // ENOMEM: can never fit
  SchedReq huge_ws;
  huge_ws.charge = 10;
  huge_ws.ws_bytes = 4096;
  CHECK(s.submit(&huge_ws, 16) == 3);        // larger than the arena
  std::vector<SchedReq> q(3);
  for (auto& r : q) {
    r.charge = 1;
    r.ws_bytes = 256;
  }
  CHECK(s.submit(&q[0], 2) == 0);
  CHECK(s.submit(&q[1], 2) == 0);
  CHECK(s.submit(&q[2], 2) == 5);            // EAGAIN: queue full
}

static void test_max_inflight_and_no_overtake() {
  FakeExec ex;
  ex.budget = 100;
  ex.lag = 2;
  Scheduler<FakeExec> s(&ex, 100, 1 << 16, 2, 0.0);
  std::vector<SchedReq> r(5);
  for (int i = 0; i < 5; ++i) {
    r[i].ticket = i + 1;
    r[i].charge = (i == 1) ? 96 : 5;   // the second one blocks on the budget
    r[i].ws_bytes = 256;
    CHECK(s.submit(&r[i], 16) == 0);
  }
  s.step();
  // only the first is admitted: #2 does not fit next to it and nobody overtakes #2
  CHECK(s.inflight() == 1);
  CHECK(s.waiting() == 4);
  int guard = 0;
  while (!s.idle() && guard++ < 100) {
    s.step();
    CHECK(s.inflight() <= 2);
  }
  CHECK(s.idle());
  for (size_t i = 1; i < ex.admit_order.size(); ++i) CHECK(ex.admit_order[i] > ex.admit_order[i - 1]);
}

static void test_watchdog() {
  FakeExec ex;
  ex.budget = 100;
  ex.cap = 1;                       // one request per launch
  Scheduler<FakeExec> s(&ex, 100, 1 << 16, 10, 0.05, /*max_retries=*/0);
  std::vector<SchedReq> r(3);
  int tag = 1;
  for (int i = 0; i < 3; ++i) {
    r[i].ticket = i + 1;
    r[i].charge = 10;
    r[i].ws_bytes = 256;
    r[i].user = (i == 1) ? &tag : nullptr;   // request 2 hangs
    CHECK(s.submit(&r[i], 16) == 0);
  }
  std::vector<SchedReq*> fin;
  const double t0 = mono_now();
  while (fin.size() < 3 && mono_now() - t0 < 2.0) {
    auto f = s.step();
    fin.insert(fin.end(), f.begin(), f.end());
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  CHECK(fin.size() == 3);
  CHECK(r[0].status == 0 && r[2].status == 0);
  CHECK(r[1].status == 4);                  // EDEVICE from the watchdog
  CHECK(s.stats().timeouts == 1);
  CHECK(s.charge_inflight() == 10);         // the hung launch keeps its memory
}

// A request that finishes before the rest of its launch is reported at
// once and frees its charge, so the next request in line is admitted while
// that launch is still open; the request that never finishes is reported by
// the watchdog and keeps its memory.
static void test_early_completion() {
  FakeExec ex;
  ex.budget = 100;
  ex.cap = 2;
  ex.lag = 1;
  Scheduler<FakeExec> s(&ex, 100, 1 << 16, 10, 0.2, /*max_retries=*/0);
  std::vector<SchedReq> r(3);
  int tag = 1;
  const size_t charge[3] = {50, 40, 50};
  for (int i = 0; i < 3; ++i) {
    r[i].ticket = 3 * (i + 1);       // ticket % 3 == 0: done after `lag` polls
    r[i].charge = charge[i];
    r[i].ws_bytes = 256;
    r[i].user = (i == 1) ? &tag : nullptr;   // request 2 never finishes
    CHECK(s.submit(&r[i], 16) == 0);
  }
  s.step();
  CHECK(s.inflight() == 2);        // 1 and 2 launched together; 3 does not fit
  CHECK(s.waiting() == 1);
  std::vector<SchedReq*> fin;
  auto f = s.step();               // 1 finishes; 3 is admitted in the same round
  fin.insert(fin.end(), f.begin(), f.end());
  CHECK(fin.size() == 1 && fin[0] == &r[0] && r[0].status == 0);
  CHECK(s.waiting() == 0);
  CHECK(s.charge_inflight() == 90);
  const double t0 = mono_now();
  while (fin.size() < 3 && mono_now() - t0 < 2.0) {
    f = s.step();
    fin.insert(fin.end(), f.begin(), f.end());
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  CHECK(fin.size() == 3);
  CHECK(r[2].status == 0);
  CHECK(r[1].status == 4);         // EDEVICE from the watchdog
  CHECK(s.stats().timeouts == 1);
  CHECK(s.charge_inflight() == 40);
  CHECK(s.stats().completed == 3);
}

// Watchdog re-admission: a request that hangs in its first launch is queued
// again at the head of the FIFO (ahead of requests submitted after it), runs
// to completion in a second launch and reports its own status; one that
// hangs every time is re-admitted once and then reported as EDEVICE.  Both
// hung launches keep their memory; the executor hears of every expiry.
static void test_watchdog_readmits() {
  FakeExec ex;
  ex.budget = 1000;
  ex.cap = 1;
  Scheduler<FakeExec> s(&ex, 1000, 1 << 16, 10, 0.05, /*max_retries=*/1);
  std::vector<SchedReq> r(4);
  int tag = 1;
  for (int i = 0; i < 4; ++i) {
    r[i].ticket = 3 * (i + 1);
    r[i].charge = 10;
    r[i].ws_bytes = 256;
  }
  ex.stuck_once.insert(r[0].ticket);   // hangs once, then runs
  r[1].user = &tag;                    // hangs every time
  for (int i = 0; i < 2; ++i) CHECK(s.submit(&r[i], 16) == 0);
  s.step();
  s.step();                            // one request per launch
  CHECK(s.inflight() == 2);
  std::vector<SchedReq*> fin;
  const double t0 = mono_now();
  bool late_submitted = false;
  while (fin.size() < 4 && mono_now() - t0 < 3.0) {
    auto f = s.step();
    fin.insert(fin.end(), f.begin(), f.end());
    if (!late_submitted && s.stats().timeouts >= 1) {
      // arrive after the first expiry: must not overtake the re-admitted ones
      for (int i = 2; i < 4; ++i) CHECK(s.submit(&r[i], 16) == 0);
      late_submitted = true;
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  }
  CHECK(fin.size() == 4);
  CHECK(r[0].status == 0 && r[0].retries == 1);
  CHECK(r[1].status == 4 && r[1].retries == 1);
  CHECK(r[2].status == 0 && r[3].status == 0);
  CHECK(s.stats().readmitted == 2);
  CHECK(s.stats().timeouts == 3);      // r0 once, r1 twice
  CHECK(ex.timeouts_seen == 3);
  // FIFO across the re-admission: r0 and r1 launched again before r2 and r3
  std::vector<uint64_t> ord = ex.admit_order;
  CHECK(ord.size() == 6);
  if (ord.size() == 6) {
    CHECK(ord[0] == r[0].ticket && ord[1] == r[1].ticket);
    CHECK(ord[2] == r[0].ticket && ord[3] == r[1].ticket);
    CHECK(ord[4] == r[2].ticket && ord[5] == r[3].ticket);
  }
  // memory of the hung launches stays reserved: r1's two launches and r0's first
  CHECK(s.charge_inflight() == 30);
}

// Requests whose inputs are not ready yet wait at the head of the FIFO and
// hold back everything behind them; once ready they run in order.
static void test_ready_gate() {
  FakeExec ex;
  ex.budget = 1000;
  ex.lag = 1;
  Scheduler<FakeExec> s(&ex, 1000, 1 << 16, 10, 0.0);
  std::vector<SchedReq> r(3);
  for (int i = 0; i < 3; ++i) {
    r[i].ticket = 3 * (i + 1);
    r[i].charge = 10;
    r[i].ws_bytes = 256;
    CHECK(s.submit(&r[i], 16) == 0);
  }
  ex.not_ready.insert(r[0].ticket);
  for (int k = 0; k < 5; ++k) s.step();
  CHECK(s.inflight() == 0 && s.waiting() == 3);
  ex.not_ready.clear();
  int guard = 0;
  while (!s.idle() && guard++ < 100) s.step();
  CHECK(s.idle());
  CHECK(ex.admit_order.size() == 3);
  for (size_t i = 1; i < ex.admit_order.size(); ++i) CHECK(ex.admit_order[i] > ex.admit_order[i - 1]);
}

// Pack construction of the server: every alignment gets exactly its W waves,
// consecutive, segments 0..W-1 in order, `first` pointing at its first wave;
// packs are full except the last of each width; bad widths and overflow are
// refused.  (A loop over a width the pack could not hold once read past the
// end of an array here.)
struct TestPack {
  int32_t inst[4];
  int16_t seg[4];
  int16_t first[4];
};

static void test_pack_by_width() {
  std::mt19937_64 rng(11);
  for (int trial = 0; trial < 200; ++trial) {
    const int n = (int)(rng() % 40);
    std::vector<int> widths(n);
    int cnt[5] = {};
    for (auto& w : widths) {
      w = 1 << (rng() % 3);
      cnt[w]++;
    }
    std::vector<TestPack> out(64);
    const int np = pack_by_width<TestPack, 4>(widths, out.data(), (int)out.size());
    CHECK(np == (cnt[4] + (cnt[2] + 1) / 2 + (cnt[1] + 3) / 4));
    std::vector<int> seen(n, 0);
    for (int p = 0; p < np; ++p) {
      for (int k = 0; k < 4; ++k) {
        const int i = out[p].inst[k];
        if (i < 0) continue;
        CHECK(i < n);
        const int W = widths[i], f = out[p].first[k];
        CHECK(out[p].seg[k] == k - f);
        CHECK(f % W == 0 && k - f < W && f + W <= 4);
        seen[i]++;
      }
    }
    for (int i = 0; i < n; ++i) CHECK(seen[i] == widths[i]);
  }
  TestPack few[2];
  CHECK((pack_by_width<TestPack, 4>({4, 4, 4}, few, 2)) == -1);   // does not fit
  CHECK((pack_by_width<TestPack, 4>({3}, few, 2)) == -1);         // 3 does not divide 4
  CHECK((pack_by_width<TestPack, 4>({8}, few, 2)) == -1);         // wider than a pack
}

static void test_arena() {
  std::mt19937_64 rng(3);
  ArenaMap a(1 << 20);
  std::vector<std::pair<size_t, size_t>> live;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 2) {
      const size_t len = 256 * (1 + rng() % 64);
      const size_t off = a.alloc(len);
      if (off != SIZE_MAX) {
        for (auto& l : live) CHECK(off + len <= l.first || l.first + l.second <= off);
        CHECK(off + len <= a.size());
        live.push_back({off, len});
      }
    } else {
      const size_t k = rng() % live.size();
      a.release(live[k].first, live[k].second);
      live.erase(live.begin() + k);
    }
  }
  for (auto& l : live) a.release(l.first, l.second);
  CHECK(a.used() == 0);
  CHECK(a.largest_free() == a.size());      // fully coalesced again
}

int main() {
  test_budget_fifo();
  test_refusals();
  test_max_inflight_and_no_overtake();
  test_watchdog();
  test_early_completion();
  test_watchdog_readmits();
  test_ready_gate();
  test_pack_by_width();
  test_arena();
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("sched ok\n");
  return 0;
}
