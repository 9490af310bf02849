// Continuous-batching scheduler for the alignment server: request FIFO,
// admission against a backpointer-memory budget, a first-fit arena, and
// completion bookkeeping.  It knows nothing about HIP: an Executor launches a
// group of admitted requests and later reports them done, so the same logic
// runs against the GPU executor (server.cpp) and a CPU fake (tests).
//
// Requests of one launch finish one by one: the executor reports each
// request's status as soon as its alignment is written, and the scheduler
// then reports it and frees its memory, without waiting for the rest of the
// launch.
//
// Admission is strictly FIFO: the oldest waiting request is admitted as soon
// as (a) its inputs are ready (the executor says so: e.g. the event its
// producer recorded has completed), (b) fewer than max_inflight requests are
// on the device, (c) its charge fits the budget next to everything in
// flight, and (d) its workspace fits a free arena range; nothing behind it
// may overtake it, so nothing starves.
// A request whose charge alone exceeds the budget is refused at submit.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <vector>

namespace ctca {

inline double mono_now() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over offsets [0, size), 256-byte granules, coalescing frees.
class ArenaMap {
 public:
  explicit ArenaMap(size_t size = 0) { reset(size); }
  void reset(size_t size) {
    free_.clear();
    size_ = size / 256 * 256;
    if (size_) free_[0] = size_;
  }
  // returns offset or SIZE_MAX
  size_t alloc(size_t len) {
    len = (len + 255) / 256 * 256;
    if (len == 0) len = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        const size_t off = it->first, rem = it->second - len;
        free_.erase(it);
        if (rem) free_[off + len] = rem;
        used_ += len;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t len) {
    len = (len + 255) / 256 * 256;
    if (len == 0) len = 256;
    used_ -= len;
    auto it = free_.emplace(off, len).first;
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
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0;
};

// Workgroup packs of kWaves waves for a group of small alignments: an
// alignment of W waves (W divides kWaves) takes W consecutive waves of a
// pack, kWaves / W alignments of one width share a pack, widest first.  Wave
// k of a pack runs segment seg[k] of alignment inst[k] (-1: idle) whose first
// wave is first[k].  Returns the number of packs written to out (at most
// cap), or -1 if a width does not divide kWaves or the packs do not fit.
template <class PackT, int kWaves>
int pack_by_width(const std::vector<int>& widths, PackT* out, int cap) {
  std::vector<std::vector<int>> by_w(kWaves + 1);
  for (size_t i = 0; i < widths.size(); ++i) {
    const int W = widths[i];
    if (W < 1 || W > kWaves || kWaves % W) return -1;
    by_w[W].push_back((int)i);
  }
  int np = 0;
  for (int W = kWaves; W >= 1; --W) {
    const std::vector<int>& v = by_w[W];
    const int per = kWaves / W;
    for (size_t i = 0; i < v.size(); i += per) {
      if (np >= cap) return -1;
      PackT& pk = out[np++];
      for (int k = 0; k < kWaves; ++k) {
        pk.inst[k] = -1;
        pk.seg[k] = 0;
        pk.first[k] = (int16_t)k;
      }
      for (int m = 0; m < per && i + m < v.size(); ++m)
        for (int k = 0; k < W; ++k) {
          pk.inst[m * W + k] = v[i + m];
          pk.seg[m * W + k] = (int16_t)k;
          pk.first[m * W + k] = (int16_t)(m * W);
        }
    }
  }
  return np;
}

struct SchedReq {
  uint64_t ticket = 0;
  size_t charge = 0;      // bytes counted against the budget
  size_t ws_bytes = 0;    // bytes taken from the arena
  size_t arena_off = SIZE_MAX;
  int status = -1;        // -1 while pending
  int retries = 0;        // re-admissions after a watchdog expiry
  double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
  void* user = nullptr;   // executor payload (descriptor of the alignment)
};

struct SchedStats {
  uint64_t submitted = 0, completed = 0, launches = 0, timeouts = 0;
  uint64_t readmitted = 0;        // requests queued again after a watchdog expiry
  size_t peak_charge = 0;
  int peak_inflight = 0;
  bool budget_violated = false;   // stays false: checked on every admission
};

template <class Exec>
class Scheduler {
 public:
  // A launch that has not finished watchdog_s seconds after it started is
  // given up on: the executor is told (on_timeout: it may restart its device
  // side), and each of its unreported requests is queued again at the head of
  // the FIFO, up to max_retries times (alignment is a pure function of its
  // inputs, so running it again is safe), then reported as EDEVICE.  The
  // launch keeps the memory of its requests until the executor reports them
  // done; a re-admitted request takes memory of its own.
  Scheduler(Exec* ex, size_t budget, size_t arena_bytes, int max_inflight, double watchdog_s,
            int max_retries = 1)
      : ex_(ex), budget_(budget), arena_(arena_bytes), max_inflight_(max_inflight),
        watchdog_s_(watchdog_s), max_retries_(max_retries) {}

  // 0 ok, 3 (ENOMEM) if the request can never fit, 5 (EAGAIN) if the queue is full
  int submit(SchedReq* r, size_t queue_cap) {
    if (r->charge > budget_ || r->ws_bytes > arena_.size()) return 3;
    if (fifo_.size() >= queue_cap) return 5;
    r->t_submit = mono_now();
    fifo_.push_back(r);
    stats_.submitted++;
    return 0;
  }

  // One scheduling round: admit what fits, launch it, retire finished
  // launches.  Returns the requests completed in this round.
  std::vector<SchedReq*> step() {
    std::vector<SchedReq*> done;
    retire(done);
    std::vector<SchedReq*> batch;
    while (!fifo_.empty() && ex_->can_launch()) {
      SchedReq* r = fifo_.front();
      if (!ex_->ready(r)) break;
      if (inflight_reqs_ >= max_inflight_) break;
      if (charge_ + r->charge > budget_) break;
      const size_t off = arena_.alloc(r->ws_bytes);
      if (off == SIZE_MAX) break;
      r->arena_off = off;
      r->t_admit = mono_now();
      charge_ += r->charge;
      if (charge_ > budget_) stats_.budget_violated = true;
      stats_.peak_charge = std::max(stats_.peak_charge, charge_);
      inflight_reqs_++;
      stats_.peak_inflight = std::max(stats_.peak_inflight, inflight_reqs_);
      fifo_.pop_front();
      batch.push_back(r);
      if ((int)batch.size() >= ex_->max_batch()) break;
    }
    if (!batch.empty()) {
      const double t = mono_now();
      for (auto* r : batch) r->t_launch = t;
      Launch L;
      L.reqs = batch;
      for (auto* r : batch) {
        L.off.push_back(r->arena_off);
        L.charge.push_back(r->charge);
        L.ws.push_back(r->ws_bytes);
      }
      L.fin.assign(batch.size(), 0);
      L.reported.assign(batch.size(), 0);
      L.t_launch = t;
      L.handle = ex_->launch(batch);
      launches_.push_back(L);
      stats_.launches++;
    }
    return done;
  }

  bool idle() const { return fifo_.empty() && launches_.empty(); }
  size_t waiting() const { return fifo_.size(); }
  int inflight() const { return inflight_reqs_; }
  size_t charge_inflight() const { return charge_; }
  const SchedStats& stats() const { return stats_; }
  const ArenaMap& arena() const { return arena_; }

 private:
  struct Launch {
    std::vector<SchedReq*> reqs;
    std::vector<size_t> off, charge, ws;   // memory of each request in this launch
    std::vector<char> fin;        // request's memory released
    std::vector<char> reported;   // request handed back (finished or timed out)
    typename Exec::Handle handle;
    double t_launch = 0;
    bool timed_out = false;
  };

  // Executor contract: ready(r) tells whether request r's inputs may be read
  // now; poll() fills st[k] with request k's status once it has
  // finished (-1 while it runs) and returns true once the whole launch is
  // over (every st[k] >= 0; its resources may then be released).
  void retire(std::vector<SchedReq*>& done) {
    for (size_t i = 0; i < launches_.size();) {
      Launch& L = launches_[i];
      std::vector<int> st;
      const bool over = ex_->poll(L.handle, L.reqs, st);
      const double t = mono_now();
      for (size_t k = 0; k < L.reqs.size(); ++k) {
        if (L.fin[k]) continue;
        int s = k < st.size() ? st[k] : -1;
        if (s < 0 && over) s = 4;   // EDEVICE: launch over without a status
        if (s < 0) continue;
        SchedReq* r = L.reqs[k];
        L.fin[k] = 1;
        arena_.release(L.off[k], L.ws[k]);
        charge_ -= L.charge[k];
        inflight_reqs_--;
        if (!L.reported[k]) {
          L.reported[k] = 1;
          r->status = s;
          r->t_done = t;
          done.push_back(r);
          stats_.completed++;
        }
      }
      if (over) {
        ex_->release(L.handle);
        launches_.erase(launches_.begin() + i);
        continue;
      }
      // watchdog: re-admit (or finally report) the requests of a launch that
      // does not finish; their memory here stays reserved until the executor
      // reports them done
      if (!L.timed_out && watchdog_s_ > 0 && t - L.t_launch > watchdog_s_) {
        L.timed_out = true;
        stats_.timeouts++;
        ex_->on_timeout(L.handle);
        std::vector<SchedReq*> again;
        for (size_t k = 0; k < L.reqs.size(); ++k) {
          if (L.reported[k]) continue;
          L.reported[k] = 1;
          SchedReq* r = L.reqs[k];
          if (r->retries < max_retries_) {
            r->retries++;
            r->arena_off = SIZE_MAX;
            stats_.readmitted++;
            again.push_back(r);
            continue;
          }
          r->status = 4;   // EDEVICE
          r->t_done = t;
          done.push_back(r);
          stats_.completed++;
        }
        // back into the FIFO at their place in submission order (ahead of
        // everything submitted after them)
        for (SchedReq* r : again) {
          auto pos = fifo_.begin();
          while (pos != fifo_.end() && (*pos)->t_submit <= r->t_submit) ++pos;
          fifo_.insert(pos, r);
        }
      }
      ++i;
    }
  }

  Exec* ex_;
  size_t budget_;
  ArenaMap arena_;
  int max_inflight_;
  double watchdog_s_;
  int max_retries_;
  std::deque<SchedReq*> fifo_;
  std::vector<Launch> launches_;
  size_t charge_ = 0;
  int inflight_reqs_ = 0;
  SchedStats stats_;
};

}  // namespace ctca
