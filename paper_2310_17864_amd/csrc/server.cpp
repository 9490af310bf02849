// Alignment server: continuous batching on one GPU.
//
// Requests (device-resident emissions and labels) are submitted from any host
// thread; a worker thread runs the Scheduler (sched.hpp): strict FIFO
// admission against the backpointer-memory budget, first-fit placement of
// each admitted request's workspace in one device arena, then the executor
// below.
//
// The executor keeps one resident kernel on the device (k_serve: a 16-wave
// workgroup per CU) instead of launching kernels per group: launches queued
// behind a running kernel on a shared hardware queue would wait for it to
// finish, so a short request could sit behind a long one.  The host turns
// each admitted group into work items (small alignments packed 16 waves to
// an item, each larger or padded one alone), keeps them in a FIFO and hands
// them to idle workgroups through per-workgroup mailboxes in fine-grained
// pinned host memory.  Each alignment raises its own completion flag there as
// soon as its outputs are written, so a request is reported (and its memory
// reused) without waiting for anything else.  The kernel is stopped after a
// short idle period and started again when work arrives.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
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

constexpr int kMaxBatch = 1024;       // requests per admitted group
constexpr int kFlags = 1 << 16;       // completion flags (requests in flight)
constexpr double kIdleStop = 0.02;    // seconds without work before the kernel is stopped
constexpr int64_t kDeviceIdle = 1000000000;  // a workgroup's own idle limit: 10 s of the 100 MHz clock
constexpr int kRegions = 16;          // sync regions: large alignments spread over workgroups at once
constexpr int kMaxDev = 64;

struct Payload {
  ctcalign_request req;
  Geo g;            // layout on one resident workgroup
  Geo gp;           // layout over several resident workgroups (W = 0: none)
  size_t bp_bytes;  // workspace part for backpointers (the larger of the two layouts)
  size_t pad_bytes; // workspace part for a padded emission copy (0 if none)
  int stride;
};

// Sync regions of multi-workgroup alignments live in uncached device memory,
// which is never freed once a kernel has read it: servers take them from a
// per-device pool and give them back.
std::mutex g_xpool_mu;
std::vector<XSync*> g_xpool[kMaxDev];

XSync* xpool_take(int dev) {
  std::lock_guard<std::mutex> lk(g_xpool_mu);
  if (!g_xpool[dev].empty()) {
    XSync* x = g_xpool[dev].back();
    g_xpool[dev].pop_back();
    return x;
  }
  void* p = nullptr;
  if (hipExtMallocWithFlags(&p, sizeof(XSync), hipDeviceMallocUncached) != hipSuccess) return nullptr;
  return static_cast<XSync*>(p);
}

void xpool_give(int dev, XSync* x) {
  std::lock_guard<std::mutex> lk(g_xpool_mu);
  g_xpool[dev].push_back(x);
}

// 16-wave pack of small alignments (pack_by_width's layout)
struct Pack16 {
  int32_t inst[kServeWaves];
  int16_t seg[kServeWaves];
  int16_t first[kServeWaves];
};

template <class T>
int host_alloc(T** h, T** d, size_t n) {
  HIP_TRY(hipHostMalloc((void**)h, sizeof(T) * n, hipHostMallocMapped | hipHostMallocCoherent));
  std::memset((void*)*h, 0, sizeof(T) * n);
  HIP_TRY(hipHostGetDevicePointer((void**)d, *h, 0));
  return CTCALIGN_OK;
}

class ServeExec {
 public:
  struct Handle {
    std::vector<int> flag;   // per request: its completion flag
  };

  ServeExec(ctcalign_ctx* ctx, char* arena) : ctx_(ctx), arena_(arena) {}

  int init() {
    // one resident workgroup per CU holds the whole device while it runs;
    // CTCALIGN_SERVE_WGS keeps it to fewer CUs (the rest stay free for
    // other kernels)
    grid_ = std::max(ctx_->num_cu, 1);
    if (const char* v = std::getenv("CTCALIGN_SERVE_WGS")) {
      const int n = std::atoi(v);
      if (n >= 1 && n < grid_) grid_ = n;
    }
    if (ctx_->device < 0 || ctx_->device >= kMaxDev) return CTCALIGN_EDEVICE;
    HIP_TRY(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&ended_, hipEventDisableTiming));
    int rc;
    if ((rc = host_alloc(&h_items_, &d_items_, grid_)) || (rc = host_alloc(&h_box_, &d_box_, grid_)) ||
        (rc = host_alloc(&h_stop_, &d_stop_, 16)) || (rc = host_alloc(&h_flag_, &d_flag_, kFlags)))
      return rc;
    sent_.assign(grid_, 0);
    busy_.assign(grid_, 0);
    idle_since_.assign(grid_, 0.0);
    reset_of_.assign(grid_, -1);
    flag_region_.assign(kFlags, -1);
    free_flag_.reserve(kFlags);
    for (int i = kFlags - 1; i >= 0; --i) free_flag_.push_back(i);
    // sync regions: each is reset by the kernel before its first use
    for (int r = 0; r < kRegions; ++r) {
      XSync* x = xpool_take(ctx_->device);
      if (!x) return CTCALIGN_ENOMEM;
      regions_.push_back(Region{x, 0, false, false});
      schedule_reset(r);
    }
    return CTCALIGN_OK;
  }

  // stops the kernel (finishing the items it runs) and frees everything
  void destroy() {
    if (h_stop_) __atomic_store_n(h_stop_, 1, __ATOMIC_RELEASE);
    if (stream_) (void)hipStreamSynchronize(stream_);
    if (ended_) (void)hipEventDestroy(ended_);
    if (stream_) (void)hipStreamDestroy(stream_);
    for (void* h : {(void*)h_items_, (void*)h_box_, (void*)h_stop_, (void*)h_flag_})
      if (h) (void)hipHostFree(h);
    for (auto& r : regions_) xpool_give(ctx_->device, r.xs);
    regions_.clear();
    h_items_ = nullptr;
    h_box_ = nullptr;
    h_stop_ = nullptr;
    h_flag_ = nullptr;
    stream_ = nullptr;
    ended_ = nullptr;
  }

  int max_batch() const { return kMaxBatch; }

  // the request's producer has finished writing its inputs
  bool ready(const SchedReq* r) const {
    const Payload* p = static_cast<const Payload*>(r->user);
    if (!p->req.ready_event) return true;
    const hipError_t e = hipEventQuery(static_cast<hipEvent_t>(p->req.ready_event));
    if (e == hipErrorNotReady) return false;
    if (e != hipSuccess) CTCA_LOG(1, "server: ready event of ticket %llu: %s",
                                  (unsigned long long)r->ticket, hipGetErrorString(e));
    return true;
  }

  // the watchdog gave up on a launch: stop the resident kernel, so that it
  // is started again (a new epoch) for the re-admitted requests once it has
  // ended
  void on_timeout(Handle&) {
    if (running_ && !stopping_) {
      stopping_ = true;
      __atomic_store_n(h_stop_, 1, __ATOMIC_RELEASE);
    }
  }

  // room for a whole group: its flags, and a bounded FIFO of items
  bool can_launch() const {
    return (int)free_flag_.size() >= kMaxBatch && (int)pending_.size() < 4 * grid_;
  }

  Handle launch(std::vector<SchedReq*>& reqs) {
    Handle h;
    h.flag.resize(reqs.size());
    std::vector<Inst> insts(reqs.size());
    std::vector<int> small;
    for (size_t k = 0; k < reqs.size(); ++k) {
      const Payload* p = static_cast<Payload*>(reqs[k]->user);
      const int f = free_flag_.back();
      free_flag_.pop_back();
      __atomic_store_n(h_flag_ + f, -1, __ATOMIC_RELEASE);
      h.flag[k] = f;
      const bool fits = (p->gp.W + kServePartWaves - 1) / kServePartWaves <= grid_;
      const int r = p->gp.W > 0 && fits ? free_region() : -1;
      if (r >= 0) {
        // over several resident workgroups, tagged with the region's next
        // generation
        Region& rg = regions_[r];
        rg.busy = true;
        ++rg.gen;
        flag_region_[f] = r;
        const Inst in = make_inst(*p, p->gp, reqs[k]->arena_off, d_flag_ + f);
        const int nparts = (in.W + kServePartWaves - 1) / kServePartWaves;
        for (int part = 0; part < nparts; ++part) {
          ServeItem it = blank_item();
          it.kind = kItemPart;
          it.inst[0] = in;
          it.xs = rg.xs;
          it.xtag = x_gen_tag(rg.gen);
          it.part = (int16_t)part;
          it.nparts = (int16_t)nparts;
          pending_.push_back(it);
        }
        continue;
      }
      insts[k] = make_inst(*p, p->g, reqs[k]->arena_off, d_flag_ + f);
      if (p->pad_bytes || p->g.W > kPackWaves) {
        ServeItem it = blank_item();
        it.inst[0] = insts[k];
        for (int w = 0; w < p->g.W; ++w) {
          it.which[w] = 0;
          it.seg[w] = (int8_t)w;
          it.first[w] = 0;
        }
        if (p->pad_bytes) {
          it.npad = 1;
          it.pad = PadDesc{p->req.emission, const_cast<float*>(insts[k].em), p->req.T, p->req.C,
                           p->stride, 0};
        }
        pending_.push_back(it);
      } else {
        small.push_back((int)k);
      }
    }
    if (!small.empty()) {
      // similar chain lengths share an item (an item holds its workgroup
      // until its longest alignment is done)
      std::sort(small.begin(), small.end(), [&](int a, int b) {
        return (int64_t)insts[a].T * insts[a].M > (int64_t)insts[b].T * insts[b].M;
      });
      std::vector<int> widths(small.size());
      for (size_t i = 0; i < small.size(); ++i) widths[i] = insts[small[i]].W;
      std::vector<Pack16> packs(small.size());
      const int np = pack_by_width<Pack16, kServeWaves>(widths, packs.data(), (int)packs.size());
      for (int q = 0; q < np; ++q) {
        ServeItem it = blank_item();
        int used = 0;
        int slot_of[kServeWaves];
        for (int w = 0; w < kServeWaves; ++w) {
          const int i = packs[q].inst[w];
          if (i < 0) continue;
          if (packs[q].seg[w] == 0) {
            slot_of[w] = used;
            it.inst[used++] = insts[small[i]];
          } else {
            slot_of[w] = slot_of[packs[q].first[w]];
          }
          it.which[w] = (int8_t)slot_of[w];
          it.seg[w] = (int8_t)packs[q].seg[w];
          it.first[w] = (int8_t)packs[q].first[w];
        }
        pending_.push_back(it);
      }
    }
    pump();
    return h;
  }

  // st[k]: request k's status once its flag is up, else -1 (EDEVICE for
  // all once the kernel could not be launched)
  bool poll(Handle& h, const std::vector<SchedReq*>& reqs, std::vector<int>& st) {
    st.assign(reqs.size(), -1);
    bool all = true;
    for (size_t k = 0; k < reqs.size(); ++k) {
      st[k] = __atomic_load_n(h_flag_ + h.flag[k], __ATOMIC_ACQUIRE);
      if (st[k] < 0 && launch_failed_ && !running_) st[k] = CTCALIGN_EDEVICE;
      if (st[k] >= 0 && flag_region_[h.flag[k]] >= 0) {
        // the top segment finishes last: the region is no longer in use
        release_region(flag_region_[h.flag[k]]);
        flag_region_[h.flag[k]] = -1;
      }
      all &= st[k] >= 0;
    }
    return all;
  }

  void release(Handle& h) {
    for (int f : h.flag) free_flag_.push_back(f);
    h.flag.clear();
  }

  // Starts or stops the kernel and hands queued items to idle workgroups.
  // Called by the worker after every scheduling round.
  void pump() {
    if (running_ && hipEventQuery(ended_) != hipErrorNotReady) {
      running_ = false;
      if (stopping_) {
        stopping_ = false;
        __atomic_store_n(h_stop_, 0, __ATOMIC_RELEASE);
      }
    }
    const bool unacked = any_unacked();
    if (!running_ && !launch_failed_ && (!pending_.empty() || unacked)) {
      ++epoch_;
      // workgroups of an earlier launch that never got to run their mailbox
      // find it again: a new launch starts from the last acknowledged item
      const bool err = launch_serve(d_items_, d_box_, d_stop_, epoch_, kDeviceIdle, grid_, stream_) !=
                           hipSuccess ||
                       hipEventRecord(ended_, stream_) != hipSuccess;
      if (err) {
        // the device no longer runs kernels: every queued and future
        // request fails (nothing of theirs can still be running)
        launch_failed_ = true;
        pending_.clear();
        return;
      }
      running_ = true;
      last_work_ = mono_now();
    }
    if (!running_ || stopping_) return;
    // idle workgroups, most recently finished first: those still poll their
    // mailbox often (a workgroup backs off the longer it idles); a finished
    // reset frees its region
    std::vector<int> idle;
    const double now = mono_now();
    for (int n = 0; n < grid_; ++n) {
      const int b = (rr_ + n) % grid_;
      const uint64_t live = __atomic_load_n(&h_box_[b].live, __ATOMIC_ACQUIRE);
      const uint64_t ack = __atomic_load_n(&h_box_[b].ack, __ATOMIC_ACQUIRE);
      if (ack != sent_[b]) continue;
      if (busy_[b]) {
        busy_[b] = 0;
        idle_since_[b] = now;
      }
      if (reset_of_[b] >= 0) {
        regions_[reset_of_[b]].gen = 0;
        regions_[reset_of_[b]].resetting = false;
        reset_of_[b] = -1;
      }
      if (live == epoch_) idle.push_back(b);
    }
    std::stable_sort(idle.begin(), idle.end(),
                     [&](int a, int b) { return idle_since_[a] > idle_since_[b]; });
    // hand out items in order; the parts of one alignment go out together
    // (they wait on each other), or not at all this round
    size_t next = 0;
    while (!pending_.empty()) {
      const ServeItem& head = pending_.front();
      const size_t unit = head.kind == kItemPart ? (size_t)head.nparts : 1;
      if (idle.size() - next < unit) break;
      bool gone = false;
      for (size_t u = 0; u < unit; ++u) {
        const int b = idle[next++];
        rr_ = (b + 1) % grid_;
        busy_[b] = 1;
        const ServeItem& it = pending_.front();
        if (it.kind == kItemReset) reset_of_[b] = region_of(it.xs);
        std::memcpy((void*)&h_items_[b], &it, sizeof(ServeItem));
        pending_.pop_front();
        ++sent_[b];
        __atomic_store_n(&h_box_[b].mail, sent_[b] << 32, __ATOMIC_RELEASE);
        // a workgroup leaving withdraws `live` before its last look at the
        // mailbox: if it is gone now, it may not have seen this item, and a
        // restarted kernel runs it
        __atomic_thread_fence(__ATOMIC_SEQ_CST);
        gone |= __atomic_load_n(&h_box_[b].live, __ATOMIC_ACQUIRE) != epoch_;
      }
      if (gone) {
        stopping_ = true;
        __atomic_store_n(h_stop_, 1, __ATOMIC_RELEASE);
        break;
      }
    }
    if (!pending_.empty() || unacked) {
      last_work_ = mono_now();
    } else if (mono_now() - last_work_ > kIdleStop) {
      stopping_ = true;
      __atomic_store_n(h_stop_, 1, __ATOMIC_RELEASE);
    }
  }

  // nothing queued or running on the device
  bool device_idle() const { return !running_ && pending_.empty(); }
  bool launch_failed() const { return launch_failed_; }

 private:
  struct Region {
    XSync* xs;
    uint32_t gen;      // generation of its last alignment since the last reset
    bool busy;         // an alignment uses it
    bool resetting;    // its reset item has not been acknowledged yet
  };

  int free_region() const {
    for (size_t r = 0; r < regions_.size(); ++r)
      if (!regions_[r].busy && !regions_[r].resetting && regions_[r].gen + 1 < (uint32_t)kXGens)
        return (int)r;
    return -1;
  }

  int region_of(const XSync* xs) const {
    for (size_t r = 0; r < regions_.size(); ++r)
      if (regions_[r].xs == xs) return (int)r;
    return -1;
  }

  // a reset item goes to the front of the queue; the region is usable again
  // once a workgroup has acknowledged it
  void schedule_reset(int r) {
    regions_[r].resetting = true;
    ServeItem it = blank_item();
    it.kind = kItemReset;
    it.xs = regions_[r].xs;
    pending_.push_front(it);
  }

  void release_region(int r) {
    regions_[r].busy = false;
    if (regions_[r].gen + 1 >= (uint32_t)kXGens) schedule_reset(r);
  }

  bool any_unacked() const {
    for (int b = 0; b < grid_; ++b)
      if (__atomic_load_n(&h_box_[b].ack, __ATOMIC_ACQUIRE) != sent_[b]) return true;
    return false;
  }

  static ServeItem blank_item() {
    ServeItem it;
    std::memset(&it, 0, sizeof(it));
    for (int w = 0; w < kServeWaves; ++w) {
      it.which[w] = -1;
      it.seg[w] = 0;
      it.first[w] = (int8_t)w;
    }
    return it;
  }

  Inst make_inst(const Payload& p, Geo g, size_t off, int32_t* notify) {
    Inst in{};
    in.T = p.req.T;
    in.C = p.req.C;
    in.L = p.req.L;
    in.blank = p.req.blank;
    in.lab = p.req.labels;
    in.path = p.req.out_path;
    in.scores = p.req.out_scores;
    in.total = p.req.out_total;
    in.status = nullptr;
    in.notify = notify;
    in.W = g.W;
    in.M = g.M;
    in.stride = p.stride;
    in.prio = 0;
    in.bp = reinterpret_cast<uint32_t*>(arena_ + off);
    in.em = p.pad_bytes ? reinterpret_cast<const float*>(arena_ + off + p.bp_bytes) : p.req.emission;
    return in;
  }

  ctcalign_ctx* ctx_;
  char* arena_;
  int grid_ = 0;
  hipStream_t stream_ = nullptr;
  hipEvent_t ended_ = nullptr;
  ServeItem *h_items_ = nullptr, *d_items_ = nullptr;
  ServeBox *h_box_ = nullptr, *d_box_ = nullptr;
  int32_t *h_stop_ = nullptr, *d_stop_ = nullptr;
  int32_t *h_flag_ = nullptr, *d_flag_ = nullptr;
  std::vector<uint64_t> sent_;       // per workgroup: sequence of the last item posted
  std::vector<int> free_flag_;
  std::deque<ServeItem> pending_;    // items waiting for an idle workgroup
  std::vector<Region> regions_;
  std::vector<int> reset_of_;        // per workgroup: region its unacknowledged reset item clears
  std::vector<char> busy_;           // per workgroup: an item posted, not yet seen acknowledged
  std::vector<double> idle_since_;   // per workgroup: when its last item was seen acknowledged
  std::vector<int> flag_region_;     // per completion flag: region its alignment uses
  uint64_t epoch_ = 0;
  int rr_ = 0;
  bool running_ = false, stopping_ = false, launch_failed_ = false;
  double last_work_ = 0;
};

}  // namespace

struct ctcalign_server {
  ctcalign_ctx* ctx = nullptr;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  size_t budget = 0;
  ServeExec* exec = nullptr;
  Scheduler<ServeExec>* sched = nullptr;
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
  // short sleeps while requests are in flight (the default slack is ~50 us)
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->stop && s->sched->idle()) break;
    std::vector<SchedReq*> done = s->sched->step();
    s->exec->pump();
    if (!done.empty()) {
      s->completed += done.size();
      s->cv_done.notify_all();
    }
    if (s->sched->idle() && s->exec->device_idle()) {
      s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
    } else if (s->sched->idle()) {
      // the kernel idles on the device: look again before stopping it
      s->cv_work.wait_for(lk, std::chrono::milliseconds(1));
    } else {
      // requests in flight: poll their flags every ~10 us (this thread's
      // timer slack is set to 1 us; a spin here would keep submitting
      // threads from the lock)
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
  s->exec = new ServeExec(ctx, static_cast<char*>(s->arena));
  rc = s->exec->init();
  if (rc) {
    s->exec->destroy();
    delete s->exec;
    (void)hipFree(s->arena);
    delete s;
    return rc;
  }
  s->sched = new Scheduler<ServeExec>(s->exec, bp_budget_bytes, s->arena_bytes, max_inflight, 30.0);
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return CTCALIGN_OK;
}

int ctcalign_server_submit(ctcalign_server* s, const ctcalign_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return CTCALIGN_EINVAL;
  if (!r->emission || !r->out_path || !r->out_scores || r->T < 1 || r->T > (1 << 30) || r->C < 1 ||
      r->C > kMaxC || r->L < 0 || (r->L > 0 && !r->labels) || r->blank < 0 || r->blank >= r->C ||
      2 * (int64_t)r->L + 1 > s->ctx->tune.max_serve_states())
    return CTCALIGN_EINVAL;
  Payload* p = new (std::nothrow) Payload();
  if (!p) return CTCALIGN_ENOMEM;
  p->req = *r;
  const int S = 2 * r->L + 1;
  p->stride = row_stride_for(r->C);
  p->g = s->ctx->tune.pick_serve(S, r->C, r->T);
  if (p->g.W == 0 || !geo_ok_top1(S, p->g.W, p->g.M) || !geometry_supported_serve(p->g.W, p->g.M)) {
    delete p;
    return CTCALIGN_EINVAL;
  }
  p->bp_bytes = round_up((size_t)bp_words(r->T, p->g.W, p->g.M) * 4, 256);
  p->pad_bytes = (r->C != p->stride || !aligned16(r->emission))
                     ? round_up((size_t)r->T * p->stride * sizeof(float), 256)
                     : 0;
  // large unpadded requests may run over several workgroups (when a sync
  // region is free at launch): the workspace holds either layout
  p->gp = Geo{0, 0};
  if (S > s->ctx->tune.max_pack_states() && !p->pad_bytes && r->T <= kXMaxT) {
    const Geo gp = s->ctx->tune.pick_serve_parts(S);
    if (gp.W > 0 && geometry_supported_serve_parts(gp.W, gp.M)) {
      p->gp = gp;
      p->bp_bytes = std::max(p->bp_bytes, round_up((size_t)bp_words(r->T, gp.W, gp.M) * 4, 256));
    }
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
  out->readmitted = st.readmitted;
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
