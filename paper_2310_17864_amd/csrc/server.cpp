// Alignment server: continuous batching on one GPU.
//
// Requests (device-resident emissions and labels) are submitted from any host
// thread; a worker thread runs the Scheduler (sched.hpp): strict FIFO
// admission against the backpointer-memory budget, first-fit placement of
// each admitted request's workspace in one device arena, and launch of the
// admitted group.  A group's small alignments (S <= 4096) run as one
// persistent pack kernel; each larger one gets its own single-instance launch.
// Every launch uses a slot of its own (stream from a pool, pinned descriptor
// buffers, status array, completion event), so groups admitted while others
// are still running overlap on the device.  Completion is observed by
// querying the slots' events; statuses come back through pinned memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ctx.hpp"
#include "kernels.hpp"
#include "sched.hpp"

using namespace ctca;

namespace {

constexpr int kSlots = 32;          // concurrent launches
constexpr int kStreams = 8;         // stream pool (default priority)
constexpr int kMaxBatch = 1024;     // requests per admitted group

struct Payload {
  ctcalign_request req;
  Geo g;
  bool pack;        // runs in the persistent pack kernel
  size_t bp_bytes;  // workspace part for backpointers
  size_t pad_bytes; // workspace part for a padded emission copy (0 if none)
  int stride;
};

struct Slot {
  bool busy = false;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  Inst* h_inst = nullptr;       // pinned
  Pack* h_pack = nullptr;       // pinned
  int32_t* h_status = nullptr;  // pinned
  int32_t* h_order = nullptr;   // pinned
  Inst* d_inst = nullptr;
  int32_t* d_order = nullptr;
  Pack* d_pack = nullptr;
  int32_t* d_status = nullptr;
  int* d_head = nullptr;
  int n = 0;
};

class HipExec {
 public:
  struct Handle {
    std::vector<int> slots;
    std::vector<std::pair<int, int>> where;   // per request: (slot, index in slot)
  };

  HipExec(ctcalign_ctx* ctx, char* arena) : ctx_(ctx), arena_(arena) {}

  int init() {
    for (int i = 0; i < kStreams; ++i) HIP_TRY(hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking));
    for (int i = 0; i < kSlots; ++i) {
      Slot& s = slots_[i];
      s.stream = streams_[i % kStreams];
      HIP_TRY(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
      HIP_TRY(hipHostMalloc((void**)&s.h_inst, sizeof(Inst) * kMaxBatch));
      HIP_TRY(hipHostMalloc((void**)&s.h_pack, sizeof(Pack) * kMaxBatch));
      HIP_TRY(hipHostMalloc((void**)&s.h_status, sizeof(int32_t) * kMaxBatch));
      HIP_TRY(hipHostMalloc((void**)&s.h_order, sizeof(int32_t) * kMaxBatch));
      HIP_TRY(hipMalloc((void**)&s.d_order, sizeof(int32_t) * kMaxBatch));
      HIP_TRY(hipMalloc((void**)&s.d_inst, sizeof(Inst) * kMaxBatch));
      HIP_TRY(hipMalloc((void**)&s.d_pack, sizeof(Pack) * kMaxBatch));
      HIP_TRY(hipMalloc((void**)&s.d_status, sizeof(int32_t) * kMaxBatch));
      HIP_TRY(hipMalloc((void**)&s.d_head, sizeof(int)));
    }
    return CTCALIGN_OK;
  }

  void destroy() {
    for (auto& st : streams_)
      if (st) (void)hipStreamSynchronize(st);
    for (auto& s : slots_) {
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.h_inst) (void)hipHostFree(s.h_inst);
      if (s.h_pack) (void)hipHostFree(s.h_pack);
      if (s.h_status) (void)hipHostFree(s.h_status);
      if (s.h_order) (void)hipHostFree(s.h_order);
      if (s.d_order) (void)hipFree(s.d_order);
      if (s.d_inst) (void)hipFree(s.d_inst);
      if (s.d_pack) (void)hipFree(s.d_pack);
      if (s.d_status) (void)hipFree(s.d_status);
      if (s.d_head) (void)hipFree(s.d_head);
      s = Slot();
    }
    for (auto& st : streams_)
      if (st) (void)hipStreamDestroy(st);
  }

  int max_batch() const { return kMaxBatch; }

  // a group needs up to (#large + 1) slots; keep a margin of half the pool
  bool can_launch() const {
    int free = 0;
    for (auto& s : slots_) free += !s.busy;
    return free > kSlots / 2;
  }

  Handle launch(std::vector<SchedReq*>& reqs) {
    Handle h;
    h.where.resize(reqs.size());
    int small_slot = -1, long_slot = -1;
    int nsmall = 0, nlong = 0;
    for (size_t k = 0; k < reqs.size(); ++k) {
      const Payload* p = static_cast<Payload*>(reqs[k]->user);
      if (p->pack) {
        if (small_slot < 0) small_slot = take_slot();
        h.where[k] = {small_slot, nsmall};
        slots_[small_slot].h_inst[nsmall] = make_inst(*p, reqs[k]->arena_off, slots_[small_slot].d_status + nsmall);
        ++nsmall;
      } else if (!p->pad_bytes) {
        // large trellis: all of this group's go to one persistent launch
        if (long_slot < 0) long_slot = take_slot();
        h.where[k] = {long_slot, nlong};
        slots_[long_slot].h_inst[nlong] = make_inst(*p, reqs[k]->arena_off, slots_[long_slot].d_status + nlong);
        ++nlong;
      } else {
        const int sl = take_slot();
        Slot& s = slots_[sl];
        s.h_inst[0] = make_inst(*p, reqs[k]->arena_off, s.d_status);
        s.n = 1;
        h.where[k] = {sl, 0};
        h.slots.push_back(sl);
        submit_one(s, *p, reqs[k]->arena_off);
      }
    }
    if (long_slot >= 0) {
      Slot& s = slots_[long_slot];
      s.n = nlong;
      h.slots.push_back(long_slot);
      submit_long(s);
    }
    if (small_slot >= 0) {
      Slot& s = slots_[small_slot];
      s.n = nsmall;
      h.slots.push_back(small_slot);
      submit_packs(s);
    }
    return h;
  }

  bool poll(Handle& h, const std::vector<SchedReq*>& reqs, std::vector<int>& st) {
    for (int sl : h.slots)
      if (hipEventQuery(slots_[sl].done) == hipErrorNotReady) return false;
    st.resize(reqs.size());
    for (size_t k = 0; k < reqs.size(); ++k) {
      const int sl = h.where[k].first;
      st[k] = launch_err_[sl] ? CTCALIGN_EDEVICE : slots_[sl].h_status[h.where[k].second];
    }
    return true;
  }

  void release(Handle& h) {
    for (int sl : h.slots) {
      slots_[sl].busy = false;
      launch_err_[sl] = false;
    }
    h.slots.clear();
  }

 private:
  int take_slot() {
    for (int i = 0; i < kSlots; ++i) {
      const int sl = (next_ + i) % kSlots;
      if (!slots_[sl].busy) {
        slots_[sl].busy = true;
        next_ = sl + 1;
        return sl;
      }
    }
    return 0;   // unreachable: can_launch() keeps half the pool free
  }

  Inst make_inst(const Payload& p, size_t off, int32_t* status) {
    Inst in{};
    in.T = p.req.T;
    in.C = p.req.C;
    in.L = p.req.L;
    in.blank = p.req.blank;
    in.lab = p.req.labels;
    in.path = p.req.out_path;
    in.scores = p.req.out_scores;
    in.total = p.req.out_total;
    in.status = status;
    in.W = p.g.W;
    in.M = p.g.M;
    in.stride = p.stride;
    in.prio = 0;
    in.bp = reinterpret_cast<uint32_t*>(arena_ + off);
    in.em = p.pad_bytes ? reinterpret_cast<const float*>(arena_ + off + p.bp_bytes) : p.req.emission;
    return in;
  }

  void pad_if_needed(const Payload& p, size_t off, hipStream_t st, bool& err) {
    if (!p.pad_bytes) return;
    const PadDesc pd{p.req.emission, reinterpret_cast<float*>(arena_ + off + p.bp_bytes), p.req.T,
                     p.req.C, p.stride, 0};
    err |= launch_pad_one(pd, st) != hipSuccess;
  }

  void submit_one(Slot& s, const Payload& p, size_t off) {
    const int sl = (int)(&s - slots_);
    bool err = false;
    pad_if_needed(p, off, s.stream, err);
    err |= launch_one(s.h_inst[0], s.stream) != hipSuccess;
    err |= hipMemcpyAsync(s.h_status, s.d_status, sizeof(int32_t), hipMemcpyDeviceToHost, s.stream) != hipSuccess;
    err |= hipEventRecord(s.done, s.stream) != hipSuccess;
    launch_err_[sl] = err;
  }

  void submit_long(Slot& s) {
    const int sl = (int)(&s - slots_);
    bool err = false;
    // longest first
    for (int i = 0; i < s.n; ++i) s.h_order[i] = i;
    std::sort(s.h_order, s.h_order + s.n, [&](int a, int b) {
      return (int64_t)s.h_inst[a].T * s.h_inst[a].M > (int64_t)s.h_inst[b].T * s.h_inst[b].M;
    });
    err |= hipMemcpyAsync(s.d_inst, s.h_inst, sizeof(Inst) * s.n, hipMemcpyHostToDevice, s.stream) != hipSuccess;
    err |= hipMemcpyAsync(s.d_order, s.h_order, sizeof(int32_t) * s.n, hipMemcpyHostToDevice, s.stream) != hipSuccess;
    err |= launch_fill(s.d_head, 1, 0, s.stream) != hipSuccess;
    const int grid = std::min(s.n, ctx_->num_cu * 4);
    err |= launch_persistent_long(s.d_inst, s.d_order, s.n, s.d_head, grid, s.stream) != hipSuccess;
    err |= hipMemcpyAsync(s.h_status, s.d_status, sizeof(int32_t) * s.n, hipMemcpyDeviceToHost, s.stream) != hipSuccess;
    err |= hipEventRecord(s.done, s.stream) != hipSuccess;
    launch_err_[sl] = err;
  }

  void submit_packs(Slot& s) {
    const int sl = (int)(&s - slots_);
    bool err = false;
    // packs of kPackWaves waves: kPackWaves / W instances of W waves each
    // (padded emissions never come here: they take a single launch with its
    // pad kernel)
    std::vector<int> by_w[kPackWaves + 1];
    for (int i = 0; i < s.n; ++i) by_w[s.h_inst[i].W].push_back(i);
    int np = 0;
    auto blank_pack = [] {
      Pack pk;
      for (int k = 0; k < kPackWaves; ++k) {
        pk.inst[k] = -1;
        pk.seg[k] = 0;
        pk.first[k] = (int16_t)k;
      }
      return pk;
    };
    for (int W : {8, 4, 2, 1}) {
      const auto& v = by_w[W];
      const int per = kPackWaves / W;
      for (size_t i = 0; i < v.size(); i += per) {
        Pack pk = blank_pack();
        for (int m = 0; m < per && i + m < v.size(); ++m)
          for (int k = 0; k < W; ++k) {
            pk.inst[m * W + k] = v[i + m];
            pk.seg[m * W + k] = (int16_t)k;
            pk.first[m * W + k] = (int16_t)(m * W);
          }
        s.h_pack[np++] = pk;
      }
    }
    err |= hipMemcpyAsync(s.d_inst, s.h_inst, sizeof(Inst) * s.n, hipMemcpyHostToDevice, s.stream) != hipSuccess;
    err |= hipMemcpyAsync(s.d_pack, s.h_pack, sizeof(Pack) * np, hipMemcpyHostToDevice, s.stream) != hipSuccess;
    err |= launch_fill(s.d_head, 1, 0, s.stream) != hipSuccess;
    const int grid = std::min(np, ctx_->num_cu * 16);
    err |= launch_persistent(s.d_inst, s.d_pack, np, s.d_head, grid, s.stream, nullptr) != hipSuccess;
    err |= hipMemcpyAsync(s.h_status, s.d_status, sizeof(int32_t) * s.n, hipMemcpyDeviceToHost, s.stream) != hipSuccess;
    err |= hipEventRecord(s.done, s.stream) != hipSuccess;
    launch_err_[sl] = err;
  }

  ctcalign_ctx* ctx_;
  char* arena_;
  hipStream_t streams_[kStreams] = {};
  Slot slots_[kSlots];
  bool launch_err_[kSlots] = {};
  int next_ = 0;
};

}  // namespace

struct ctcalign_server {
  ctcalign_ctx* ctx = nullptr;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  size_t budget = 0;
  HipExec* exec = nullptr;
  Scheduler<HipExec>* sched = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  size_t queue_cap = 1 << 20;
  std::unordered_map<uint64_t, SchedReq*> reqs;
  std::atomic<uint64_t> completed{0};
};

namespace {

void worker_loop(ctcalign_server* s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->stop && s->sched->idle()) break;
    std::vector<SchedReq*> done = s->sched->step();
    if (!done.empty()) {
      s->completed += done.size();
      s->cv_done.notify_all();
    }
    if (s->sched->idle()) {
      s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
    } else {
      // launches in flight: poll their events every few microseconds
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(10));
      lk.lock();
    }
  }
}

size_t charge_of(int32_t T, int32_t L) {
  // the budget counts 2-bit backpointers for every state and frame
  return (size_t)T * (size_t)(2 * (int64_t)L + 1) / 4 + 1;
}

}  // namespace

extern "C" {

int ctcalign_server_create(ctcalign_ctx* ctx, size_t bp_budget_bytes, int32_t max_inflight,
                           ctcalign_server** out) {
  if (!ctx || !out || bp_budget_bytes == 0 || max_inflight < 1) return CTCALIGN_EINVAL;
  *out = nullptr;
  HIP_TRY(hipSetDevice(ctx->device));
  ctcalign_server* s = new (std::nothrow) ctcalign_server();
  if (!s) return CTCALIGN_ENOMEM;
  s->ctx = ctx;
  s->budget = bp_budget_bytes;
  // workspaces (1.5-bit backpointers + padded copies) fit in the budget plus
  // a margin for padding of small trellises
  size_t freeb = 0, totalb = 0;
  (void)hipMemGetInfo(&freeb, &totalb);
  s->arena_bytes = std::min(bp_budget_bytes + bp_budget_bytes / 4 + ((size_t)64 << 20), freeb / 2);
  s->arena_bytes = round_up(s->arena_bytes, 256);
  int rc = map_hip(hipMalloc(&s->arena, s->arena_bytes), "server arena");
  if (rc) {
    delete s;
    return rc;
  }
  s->exec = new HipExec(ctx, static_cast<char*>(s->arena));
  rc = s->exec->init();
  if (rc) {
    s->exec->destroy();
    delete s->exec;
    (void)hipFree(s->arena);
    delete s;
    return rc;
  }
  s->sched = new Scheduler<HipExec>(s->exec, bp_budget_bytes, s->arena_bytes, max_inflight, 30.0);
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return CTCALIGN_OK;
}

int ctcalign_server_submit(ctcalign_server* s, const ctcalign_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return CTCALIGN_EINVAL;
  if (!r->emission || !r->out_path || !r->out_scores || r->T < 1 || r->T > (1 << 30) || r->C < 1 ||
      r->C > kMaxC || r->L < 0 || (r->L > 0 && !r->labels) || r->blank < 0 || r->blank >= r->C ||
      2 * (int64_t)r->L + 1 > kMaxS)
    return CTCALIGN_EINVAL;
  Payload* p = new (std::nothrow) Payload();
  if (!p) return CTCALIGN_ENOMEM;
  p->req = *r;
  const int S = 2 * r->L + 1;
  p->stride = row_stride_for(r->C);
  if (S <= s->ctx->tune.max_pack_states()) {
    p->g = s->ctx->tune.pick_pack(S, r->C, r->T);
    p->pack = true;
  } else {
    p->g = s->ctx->tune.pick_long(S);
    p->pack = false;
  }
  if (p->g.W == 0 || !geo_ok(S, p->g.W, p->g.M)) {
    delete p;
    return CTCALIGN_EINVAL;
  }
  p->bp_bytes = round_up((size_t)bp_words(r->T, p->g.W, p->g.M) * 4, 256);
  p->pad_bytes = (r->C != p->stride || !aligned16(r->emission))
                     ? round_up((size_t)r->T * p->stride * sizeof(float), 256)
                     : 0;
  if (p->pad_bytes && p->pack) {
    // padded emissions go through a single launch (its pad kernel runs on the same stream)
    p->pack = false;
    p->g = s->ctx->tune.pick_long(S);
    p->bp_bytes = round_up((size_t)bp_words(r->T, p->g.W, p->g.M) * 4, 256);
  }
  SchedReq* q = new (std::nothrow) SchedReq();
  if (!q) {
    delete p;
    return CTCALIGN_ENOMEM;
  }
  q->user = p;
  q->ws_bytes = p->bp_bytes + p->pad_bytes;
  q->charge = std::max(charge_of(r->T, r->L), q->ws_bytes);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    delete p;
    delete q;
    return CTCALIGN_EINVAL;
  }
  q->ticket = s->next_ticket;
  const int rc = s->sched->submit(q, s->queue_cap);
  if (rc) {
    delete p;
    delete q;
    return rc;
  }
  s->next_ticket++;
  s->reqs[q->ticket] = q;
  *ticket = q->ticket;
  s->cv_work.notify_one();
  return CTCALIGN_OK;
}

static int finish(ctcalign_server* s, uint64_t ticket, int32_t* status, ctcalign_timing* t, bool block) {
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return CTCALIGN_EINVAL;
  SchedReq* q = it->second;
  if (q->status < 0) {
    if (!block) return CTCALIGN_EBUSY;
    s->cv_done.wait(lk, [&] { return q->status >= 0; });
  }
  if (status) *status = q->status;
  if (t) {
    t->submit_s = q->t_submit;
    t->admit_s = q->t_admit;
    t->launch_s = q->t_launch;
    t->done_s = q->t_done;
  }
  // a request reported by the watchdog keeps its record (the device may still
  // write its workspace); every other record is released here
  if (q->status != CTCALIGN_EDEVICE) {
    delete static_cast<Payload*>(q->user);
    delete q;
  }
  s->reqs.erase(it);
  return CTCALIGN_OK;
}

int ctcalign_server_poll(ctcalign_server* s, uint64_t ticket, int32_t* status, ctcalign_timing* t) {
  if (!s) return CTCALIGN_EINVAL;
  return finish(s, ticket, status, t, false);
}

int ctcalign_server_wait(ctcalign_server* s, uint64_t ticket, int32_t* status, ctcalign_timing* t) {
  if (!s) return CTCALIGN_EINVAL;
  return finish(s, ticket, status, t, true);
}

int ctcalign_server_get_stats(ctcalign_server* s, ctcalign_server_stats* out) {
  if (!s || !out) return CTCALIGN_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const SchedStats& st = s->sched->stats();
  out->submitted = st.submitted;
  out->completed = st.completed;
  out->launches = st.launches;
  out->timeouts = st.timeouts;
  out->peak_charge_bytes = st.peak_charge;
  out->budget_bytes = s->budget;
  out->peak_inflight = st.peak_inflight;
  out->waiting = (int32_t)s->sched->waiting();
  out->inflight = s->sched->inflight();
  out->budget_violated = st.budget_violated ? 1 : 0;
  return CTCALIGN_OK;
}

int ctcalign_server_destroy(ctcalign_server* s) {
  if (!s) return CTCALIGN_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  s->exec->destroy();
  for (auto& kv : s->reqs) {
    delete static_cast<Payload*>(kv.second->user);
    delete kv.second;
  }
  delete s->sched;
  delete s->exec;
  (void)hipSetDevice(s->ctx->device);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
  return CTCALIGN_OK;
}

}  // extern "C"
