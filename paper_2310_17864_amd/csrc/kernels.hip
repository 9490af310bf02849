// gfx950 kernels for CTC forced alignment and their host-side launchers.
//
//   k_one                one instance, W <= 4 waves, M <= 16 states per lane
//   k_one_long           one instance, W <= 8 waves, 16 <= M <= 64 (long form)
//   k_persistent         batched: each 4-wave workgroup pops work items
//                        ("packs") from a device queue until it is empty
//   k_fill               small fill kernel (queue reset inside graphs)
//
// Emission rows sit in LDS with a stride of 256 floats; in HBM their stride
// is 32 (C <= 32) or 256 (32 < C <= 256), padded by the host when needed.
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "kernels.hpp"

namespace ctca {

// Runs segment w of `in` on the calling wave: label check, one workgroup
// barrier, forward pass, then either "done" publication (lower segments) or
// end-state selection and backtrack (the top segment).
template <int M>
__device__ __forceinline__ void run_wave(const Inst& in, int w, int lane, SegSync* sy, const Ring& ring) {
  const bool bad = prologue_check<M>(in, w, lane);
  if (bad && lane == 0) sy[w].bad = 1;
  __syncthreads();
  bool any_bad = false;
  for (int k = 0; k < in.W; ++k) any_bad |= (sy[k].bad != 0);
  const FwdOut fo = segment_forward<M>(in, w, lane, ring, sy, any_bad);
  if (w + 1 < in.W) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // backpointer stores reach L2
    if (lane == 0) lds_store_rel(&sy[w].done, 1);
  } else {
    bool ok = fo.ok != 0;
    for (int k = 0; k + 1 < in.W; ++k) ok &= wait_geq(&sy[k].done, 1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    FwdOut f2 = fo;
    f2.ok = ok ? 1 : 0;
    backtrack<M>(in, f2, any_bad ? kEinval : kOk, lane);
  }
}

__device__ __forceinline__ void set_prio(int p) {
  switch (p) {
    case 3: __builtin_amdgcn_s_setprio(3); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    default: __builtin_amdgcn_s_setprio(0); break;
  }
}

__device__ __forceinline__ void reset_sync(SegSync* s, int lane) {
  if (lane == 0) {
    s->prod = 0;
    s->cons = 0;
    s->done = 0;
    s->bad = 0;
  }
}

#define CTCA_CASE(MM) \
  case MM:            \
    run_wave<MM>(in, w, lane, sy, Ring{ring[w]}); \
    break;

// LDS of the single-instance kernels: per wave a SegSync and an 8-row
// emission ring.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_one(Inst in) {
  __shared__ SegSync sy[4];
  __shared__ __attribute__((aligned(16))) float ring[4][kRing * kMaxC];
  // the wave index is uniform across a wave; readfirstlane tells the compiler
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  reset_sync(sy + w, lane);
  switch (in.M) {
    CTCA_CASE(2) CTCA_CASE(4) CTCA_CASE(6) CTCA_CASE(8)
    CTCA_CASE(10) CTCA_CASE(12) CTCA_CASE(14) CTCA_CASE(16)
    default: __syncthreads(); break;
  }
}

// Long form: up to 8 waves (2 per SIMD), up to 64 states per lane.
__global__ void __launch_bounds__(512) k_one_long(Inst in) {
  __shared__ SegSync sy[8];
  __shared__ __attribute__((aligned(16))) float ring[8][kRing * kMaxC];
  // the wave index is uniform across a wave; readfirstlane tells the compiler
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  reset_sync(sy + w, lane);
  switch (in.M) {
    CTCA_CASE(16) CTCA_CASE(24) CTCA_CASE(32) CTCA_CASE(40)
    CTCA_CASE(48) CTCA_CASE(56) CTCA_CASE(60) CTCA_CASE(64)
    default: __syncthreads(); break;
  }
}

__device__ __forceinline__ void pack_dispatch(const Inst& in, int w, int lane, SegSync* sy,
                                              const Ring& r) {
  switch (in.M) {
    case 2: run_wave<2>(in, w, lane, sy, r); break;
    case 4: run_wave<4>(in, w, lane, sy, r); break;
    case 6: run_wave<6>(in, w, lane, sy, r); break;
    case 8: run_wave<8>(in, w, lane, sy, r); break;
    case 10: run_wave<10>(in, w, lane, sy, r); break;
    case 12: run_wave<12>(in, w, lane, sy, r); break;
    case 14: run_wave<14>(in, w, lane, sy, r); break;
    case 16: run_wave<16>(in, w, lane, sy, r); break;
    default: __syncthreads(); break;
  }
}

// LDS: 4 SegSync and, per wave, an 8-row emission ring of the widest stride.
// trace (optional, may be null): per pack {start, end} of the 100 MHz
// wall clock and the hardware id of the CU that ran it.
__global__ void __launch_bounds__(kWave * kPackWaves) __attribute__((amdgpu_waves_per_eu(4))) k_persistent(const Inst* __restrict__ insts,
                                                    const Pack* __restrict__ packs, int npacks,
                                                    int* __restrict__ head,
                                                    int64_t* __restrict__ trace) {
  __shared__ SegSync sy[kPackWaves];
  __shared__ __attribute__((aligned(16))) float ring[kPackWaves][kRing * kMaxC];
  __shared__ int s_item;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(head, 1);
    reset_sync(sy + wv, lane);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= npacks) break;
    if (trace && threadIdx.x == 0) {
      trace[3 * item] = (int64_t)__builtin_amdgcn_s_memrealtime();
      trace[3 * item + 2] = (int64_t)__builtin_amdgcn_s_getreg((4 << 0) | (0 << 6) | (31 << 11));
    }
    const int ii = packs[item].inst[wv];
    if (ii < 0) {
      __syncthreads();   // the barrier the busy waves take inside run_wave
    } else {
      const Inst in = insts[ii];
      const int seg = packs[item].seg[wv];
      const int first = packs[item].first[wv];
      set_prio(in.prio);
      pack_dispatch(in, seg, lane, sy + first, Ring{ring[wv]});
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();     // every wave is done with this pack's LDS
    if (trace && threadIdx.x == 0) trace[3 * item + 1] = (int64_t)__builtin_amdgcn_s_memrealtime();
  }
}

// Copies rows of a [T][C] emission into a [T][stride] buffer (zeros in the
// pad columns), so the alignment kernels always see 16-byte aligned rows of
// a compiled stride.  blockIdx.y selects the descriptor.
// Batched large alignments: each 8-wave workgroup pops one instance index
// (into `order`) at a time and runs its W <= 8 segments; waves beyond W wait
// at the two workgroup barriers.  Same engine and LDS layout as k_one_long.
__global__ void __launch_bounds__(512) k_persistent_long(const Inst* __restrict__ insts,
                                                         const int* __restrict__ order, int n,
                                                         int* __restrict__ head) {
  __shared__ SegSync sy[8];
  __shared__ __attribute__((aligned(16))) float ring[8][kRing * kMaxC];
  __shared__ int s_item;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(head, 1);
    reset_sync(sy + w, lane);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(s_item);
    if (item >= n) break;
    const Inst in = insts[order[item]];
    if (w >= in.W) {
      __syncthreads();   // the barrier the busy waves take inside run_wave
    } else {
      switch (in.M) {
        CTCA_CASE(16) CTCA_CASE(24) CTCA_CASE(32) CTCA_CASE(40)
        CTCA_CASE(48) CTCA_CASE(56) CTCA_CASE(60) CTCA_CASE(64)
        default: __syncthreads(); break;
      }
    }
    __syncthreads();
  }
}

// The longest chains of a batch: one alignment per 8-wave workgroup with few
// states per lane (lower per-frame latency than a 4-wave pack), register
// budget of 4 waves per SIMD so packs of the main kernel share the CU.  One
// workgroup per alignment (no queue): the plan launches at most one per CU,
// on a parallel branch of its graph, before the pack kernel.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_persistent_crit(const Inst* __restrict__ insts, const int* __restrict__ order, int n) {
  __shared__ SegSync sy[8];
  __shared__ __attribute__((aligned(16))) float ring[8][kRing * kMaxC];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int item = blockIdx.x;
  if (item >= n) return;
  const Inst in = insts[order[item]];
  if (w >= in.W) {
    __syncthreads();   // the barrier the busy waves take inside run_wave
    return;
  }
  reset_sync(sy + w, lane);
  set_prio(in.prio);
  switch (in.M) {
    CTCA_CASE(4) CTCA_CASE(6) CTCA_CASE(8) CTCA_CASE(10) CTCA_CASE(12)
    default: __syncthreads(); break;
  }
}

#undef CTCA_CASE

// ---- multi layout: one long alignment over several workgroups ---------------

__device__ __forceinline__ bool wait_eq_sys(const int* p, int want) {
  for (int n = 0; n < kXSpinLimit; ++n) {
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == want) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

// Segment w = g * kWG + wl of a multi-workgroup alignment on wave wl of
// workgroup g (kWG waves per workgroup; sy[kWG] holds the incoming copy).
template <int M, int kWG>
__device__ __forceinline__ void run_multi(const Inst& in, XSync* xs, uint32_t tag, SegSync* sy,
                                          const Ring& ring, int g, int wl, int lane, bool bad) {
  const int w = g * kWG + wl;
  if (w >= in.W) return;
  XLink xl;
  xl.wl = wl;
  xl.tag = tag;
  xl.in_lds = sy + kWG;
  if (wl == 0 && g > 0) xl.in_ch = &xs->ch[g - 1];
  if (wl == kWG - 1 && w + 1 < in.W) xl.out_ch = &xs->ch[g];
  const FwdOut fo = segment_forward<M, true>(in, w, lane, ring, sy, bad, xl);
  if (w + 1 < in.W) {
    // backpointers visible device-wide, then the flag
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0)
      __hip_atomic_store(&xs->done[w], (int)(tag | 1u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  } else {
    bool ok = fo.ok != 0;
    for (int k = 0; k + 1 < in.W; ++k) ok &= wait_eq_sys(&xs->done[k], (int)(tag | 1u));
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    FwdOut f2 = fo;
    f2.ok = ok ? 1 : 0;
    backtrack<M>(in, f2, bad ? kEinval : kOk, lane);
  }
}

// Workgroup g runs segments 8g .. 8g+7 of one alignment; all workgroups are
// resident together (one launch of at most kXMaxGroups workgroups).  Every
// workgroup validates the whole transcript itself, so the verdict needs no
// communication between workgroups.  `tag` marks every word this launch
// writes to the sync region.
__global__ void __launch_bounds__(kWave * kXWaves) k_multi(Inst in, XSync* xs, uint32_t tag) {
  __shared__ SegSync sy[kXWaves + 1];   // + the copy of the incoming boundary
  __shared__ __attribute__((aligned(16))) float ring[kXWaves][kRing * kMaxC];
  const int wl = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  reset_sync(sy + wl, lane);
  if (wl == 0) reset_sync(sy + kXWaves, lane);
  bool bad = false;
  for (int i = threadIdx.x; i < in.L; i += blockDim.x) {
    const int v = in.lab[i];
    bad |= (v < 0) | (v >= in.C) | (v == in.blank);
  }
  bad = __syncthreads_or(bad);
  const int g = blockIdx.x;
  const Ring r{ring[wl]};
  switch (in.M) {
    case 2: run_multi<2, kXWaves>(in, xs, tag, sy, r, g, wl, lane, bad); break;
    case 4: run_multi<4, kXWaves>(in, xs, tag, sy, r, g, wl, lane, bad); break;
    case 6: run_multi<6, kXWaves>(in, xs, tag, sy, r, g, wl, lane, bad); break;
    case 8: run_multi<8, kXWaves>(in, xs, tag, sy, r, g, wl, lane, bad); break;
    case 10: run_multi<10, kXWaves>(in, xs, tag, sy, r, g, wl, lane, bad); break;
    case 12: run_multi<12, kXWaves>(in, xs, tag, sy, r, g, wl, lane, bad); break;
    case 14: run_multi<14, kXWaves>(in, xs, tag, sy, r, g, wl, lane, bad); break;
    case 16: run_multi<16, kXWaves>(in, xs, tag, sy, r, g, wl, lane, bad); break;
    default: break;
  }
}

// ---- resident serving kernel -------------------------------------------------

// Loads from fine-grained host memory at system scope: never served from a
// device cache, so a mailbox or an item the host rewrote is read fresh.
__device__ __forceinline__ uint64_t host_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void host_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// An LDS copy of an Inst as wave-uniform values (scalar registers), so the
// 24 words of the descriptor do not occupy vector registers.
__device__ __forceinline__ Inst uniform_inst(const Inst* src) {
  constexpr int n = sizeof(Inst) / 4;
  int v[n];
  const int* s = reinterpret_cast<const int*>(src);
#pragma unroll
  for (int k = 0; k < n; ++k) v[k] = __builtin_amdgcn_readfirstlane(s[k]);
  Inst in;
  __builtin_memcpy(&in, v, sizeof(Inst));
  return in;
}

constexpr uint64_t kServeIdle = ~0ull, kServeExit = ~0ull - 1;

// Workgroup b serves the mailbox box[b]: when its sequence number moves past
// the last one finished, the workgroup copies items[b] into LDS, pads the
// emission rows if asked, runs the item's segments (one per wave, the same
// per-wave engine as the batched kernel), and stores the sequence number
// into ack.  Each alignment raises its own completion flag as it finishes.
// Exits when the host sets *stop, or after idle_limit ticks of the 100 MHz
// clock without work.
__global__ void __launch_bounds__(kWave * kServeWaves)
k_serve(const ServeItem* items, ServeBox* box, const int32_t* stop, uint64_t epoch, int64_t idle_limit) {
  __shared__ SegSync sy[kServeWaves + 1];   // + the incoming copy of a multi-workgroup part
  __shared__ __attribute__((aligned(16))) float ring[kServeWaves][kRing * kMaxC];
  __shared__ uint64_t s_item[sizeof(ServeItem) / 8];
  __shared__ uint64_t s_cmd;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  ServeBox* bx = box + blockIdx.x;
  uint64_t done_seq = 0;                // meaningful in thread 0 only
  if (tid == 0) {
    done_seq = host_load(&bx->ack);
    host_store(&bx->live, epoch);
  }
  int64_t idle0 = (int64_t)__builtin_amdgcn_s_memrealtime();
  int idle_polls = 0;
  for (;;) {
    if (tid == 0) {
      uint64_t seq = host_load(&bx->mail) >> 32;
      uint64_t cmd = kServeIdle;
      if (seq != done_seq) {
        cmd = seq;
      } else if (__hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0 ||
                 (int64_t)__builtin_amdgcn_s_memrealtime() - idle0 > idle_limit) {
        // leave: withdraw `live`, then look at the mailbox once more.  The
        // host posts, then reads `live`; with both sides storing before
        // loading, an item posted now is either seen here or the host sees
        // this workgroup gone (and restarts the kernel).
        host_store(&bx->live, 0);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "");
        seq = host_load(&bx->mail) >> 32;
        if (seq != done_seq) {
          host_store(&bx->live, epoch);
          cmd = seq;
        } else {
          cmd = kServeExit;
        }
      }
      s_cmd = cmd;
    }
    __syncthreads();
    const uint64_t cmd = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(s_cmd >> 32)) << 32) |
                         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)s_cmd);
    __syncthreads();                    // every wave has read s_cmd
    if (cmd == kServeExit) break;
    if (cmd == kServeIdle) {
      // back off: ~3.4 us per s_sleep 127 at 2.4 GHz, up to ~55 us per poll
      const int n = 1 + (idle_polls < 120 ? idle_polls / 8 : 15);
      for (int k = 0; k < n; ++k) __builtin_amdgcn_s_sleep(127);
      ++idle_polls;
      continue;
    }
    // the item was written before its mailbox: read it after the mailbox
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    const uint64_t* src = reinterpret_cast<const uint64_t*>(items + blockIdx.x);
    for (int k = tid; k < (int)(sizeof(ServeItem) / 8); k += kWave * kServeWaves) s_item[k] = host_load(src + k);
    reset_sync(sy + w, lane);
    if (w == 0) reset_sync(sy + kServeWaves, lane);
    __syncthreads();
    const ServeItem* it = reinterpret_cast<const ServeItem*>(s_item);
    const int kind = __builtin_amdgcn_readfirstlane(it->kind);
    if (kind == kItemReset) {
      // a tag no alignment uses, in every word of the sync region
      int* p = reinterpret_cast<int*>(it->xs);
      for (int i = tid; i < (int)(sizeof(XSync) / sizeof(int)); i += kWave * kServeWaves) p[i] = -1;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    } else if (kind == kItemPart) {
      // one workgroup of a multi-workgroup alignment: every part checks the
      // whole transcript, so the verdict needs no exchange
      const Inst in = uniform_inst(&it->inst[0]);
      bool bad = false;
      for (int i = tid; i < in.L; i += kWave * kServeWaves) {
        const int v = in.lab[i];
        bad |= (v < 0) | (v >= in.C) | (v == in.blank);
      }
      bad = __syncthreads_or(bad);
      const int part = __builtin_amdgcn_readfirstlane((int)it->part);
      XSync* xs = it->xs;
      const uint32_t tag = (uint32_t)__builtin_amdgcn_readfirstlane((int)it->xtag);
      // 8 segments per workgroup (2 waves per SIMD: the chain's frames stay
      // short); waves 8..15 idle
      const Ring r{ring[w]};
      if (w < kServePartWaves) {
        switch (in.M) {
          case 4: run_multi<4, kServePartWaves>(in, xs, tag, sy, r, part, w, lane, bad); break;
          case 6: run_multi<6, kServePartWaves>(in, xs, tag, sy, r, part, w, lane, bad); break;
          case 8: run_multi<8, kServePartWaves>(in, xs, tag, sy, r, part, w, lane, bad); break;
          default: break;
        }
      }
    } else if (__builtin_amdgcn_readfirstlane(it->npad)) {
      // emission rows into the compiled stride (zeros in the pad columns)
      const PadDesc pd = it->pad;
      const int64_t n = (int64_t)pd.T * pd.stride;
      for (int64_t i = tid; i < n; i += kWave * kServeWaves) {
        const int64_t t = i / pd.stride;
        const int c = (int)(i - t * pd.stride);
        pd.dst[i] = c < pd.C ? pd.src[t * pd.C + c] : 0.f;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (kind == kItemSegments) {
      const int wi = __builtin_amdgcn_readfirstlane((int)it->which[w]);
      if (wi < 0) {
        __syncthreads();   // the barrier the busy waves take inside run_wave
      } else {
        const Inst in = uniform_inst(&it->inst[wi]);
        const int seg = __builtin_amdgcn_readfirstlane((int)it->seg[w]);
        const int first = __builtin_amdgcn_readfirstlane((int)it->first[w]);
        pack_dispatch(in, seg, lane, sy + first, Ring{ring[w]});
      }
    }
    __syncthreads();                    // the item's LDS is free again
    if (tid == 0) {
      done_seq = cmd;
      host_store(&bx->ack, cmd);
    }
    idle0 = (int64_t)__builtin_amdgcn_s_memrealtime();
    idle_polls = 0;
  }
}


__global__ void __launch_bounds__(256) k_pad(const PadDesc* __restrict__ d) {
  const PadDesc pd = d[blockIdx.y];
  const int64_t total = (int64_t)pd.T * pd.stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / pd.stride;
    const int c = (int)(i - r * pd.stride);
    pd.dst[i] = c < pd.C ? pd.src[r * pd.C + c] : 0.0f;
  }
}

__global__ void __launch_bounds__(256) k_pad_one(PadDesc pd) {
  const int64_t total = (int64_t)pd.T * pd.stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / pd.stride;
    const int c = (int)(i - r * pd.stride);
    pd.dst[i] = c < pd.C ? pd.src[r * pd.C + c] : 0.0f;
  }
}

// Token spans of a frame path: a span starts at a non-blank frame whose
// class differs from the previous frame's; its index is the number of starts
// before it (wave ballot + popcount, then a prefix over the 16 waves in LDS);
// the starting thread walks the span and folds its scores in frame order.
__global__ void __launch_bounds__(1024) k_spans(const int32_t* __restrict__ path,
                                                const float* __restrict__ scores, int T, int blank,
                                                int max_spans, int32_t* __restrict__ tok,
                                                int32_t* __restrict__ start, int32_t* __restrict__ end,
                                                float* __restrict__ score, int32_t* __restrict__ count) {
  __shared__ int wave_tot[16];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < T; c0 += 1024) {
    const int t = c0 + tid;
    int cls = -1;
    bool is_start = false;
    if (t < T) {
      cls = path[t];
      is_start = cls >= 0 && cls != blank && (t == 0 || path[t - 1] != cls);
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(is_start);
    const int before = __builtin_popcountll(m & ((lane ? (~0ull >> (64 - lane)) : 0ull)));
    if (lane == 0) wave_tot[wv] = __builtin_popcountll(m);
    __syncthreads();
    int off = base, tot = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      if (k < wv) off += wave_tot[k];
      tot += wave_tot[k];
    }
    if (is_start) {
      const int idx = off + before;
      int e = t;
      float acc = scores[t];
      while (e + 1 < T && path[e + 1] == cls) {
        ++e;
        acc = acc + scores[e];
      }
      if (idx < max_spans) {
        tok[idx] = cls;
        start[idx] = t;
        end[idx] = e + 1;
        score[idx] = acc;
      }
    }
    __syncthreads();
    if (tid == 0) base += tot;
    __syncthreads();
  }
  if (tid == 0) *count = base;
}

__global__ void k_fill(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- launchers ---------------------------------------------------------------

static bool m_in(int M, const int* menu, int n) {
  for (int i = 0; i < n; ++i)
    if (menu[i] == M) return true;
  return false;
}

static const int kOneMenu[] = {2, 4, 6, 8, 10, 12, 14, 16};
static const int kLongMenu[] = {16, 24, 32, 40, 48, 56, 60, 64};
static const int kPackMenuK[] = {2, 4, 6, 8, 10, 12, 14, 16};

static const int kMultiMenu[] = {2, 4, 6, 8, 10, 12, 14, 16};

bool geometry_supported_one(int W, int M) {
  if (W >= 1 && W <= 4 && m_in(M, kOneMenu, 8)) return true;
  if (geometry_is_multi(W, M) && W <= kXWaves * kXMaxGroups && m_in(M, kMultiMenu, 8)) return true;
  if (W >= 1 && W <= 8 && m_in(M, kLongMenu, 8)) return true;
  return false;
}

bool geometry_supported_pack(int W, int M) {
  return (W == 1 || W == 2 || W == 4 || W == 8) && W <= kPackWaves && m_in(M, kPackMenuK, 8);
}

hipError_t launch_one(const Inst& in, hipStream_t st) {
  const dim3 block(kWave * in.W);
  if (in.W <= 4 && m_in(in.M, kOneMenu, 8))
    hipLaunchKernelGGL(k_one, dim3(1), block, 0, st, in);
  else
    hipLaunchKernelGGL(k_one_long, dim3(1), block, 0, st, in);
  return hipGetLastError();
}

hipError_t launch_multi_reset(XSync* xs, hipStream_t st) {
  // every slot, count and flag -1: a tag no launch uses
  const int nwords = (int)(sizeof(XSync) / sizeof(int));
  hipLaunchKernelGGL(k_fill, dim3((nwords + 255) / 256), dim3(256), 0, st, reinterpret_cast<int*>(xs),
                     nwords, -1);
  return hipGetLastError();
}

hipError_t launch_multi(const Inst& in, XSync* xs, uint32_t gen, hipStream_t st) {
  if (gen < 1 || gen >= (uint32_t)kXGens || in.T > kXMaxT) return hipErrorInvalidValue;
  const int groups = (in.W + kXWaves - 1) / kXWaves;
  // the workgroups wait on each other: a cooperative launch guarantees they
  // are all resident at once (or fails instead of starting)
  Inst in_copy = in;
  XSync* xs_copy = xs;
  uint32_t tag = x_gen_tag(gen);
  void* args[] = {&in_copy, &xs_copy, &tag};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_multi), dim3(groups),
                                    dim3(kWave * kXWaves), args, 0, st);
}

hipError_t launch_persistent(const Inst* d_insts, const Pack* d_packs, int npacks, int* d_head,
                             int grid, hipStream_t st, int64_t* d_trace) {
  hipLaunchKernelGGL(k_persistent, dim3(grid), dim3(kWave * kPackWaves), 0, st, d_insts, d_packs,
                     npacks, d_head, d_trace);
  return hipGetLastError();
}

hipError_t launch_pad(const PadDesc* d_desc, int n, int64_t max_elems, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t bx = (max_elems + 255) / 256;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_pad, dim3((unsigned)bx, (unsigned)n), dim3(256), 0, st, d_desc);
  return hipGetLastError();
}

hipError_t launch_pad_one(const PadDesc& pd, hipStream_t st) {
  int64_t bx = ((int64_t)pd.T * pd.stride + 255) / 256;
  bx = bx > 1024 ? 1024 : (bx < 1 ? 1 : bx);
  hipLaunchKernelGGL(k_pad_one, dim3((unsigned)bx), dim3(256), 0, st, pd);
  return hipGetLastError();
}

hipError_t launch_persistent_long(const Inst* d_insts, const int* d_order, int n, int* d_head,
                                  int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_persistent_long, dim3(grid), dim3(kWave * 8), 0, st, d_insts, d_order, n,
                     d_head);
  return hipGetLastError();
}

static const int kCritMenu[] = {4, 6, 8, 10, 12};
bool geometry_supported_crit(int W, int M) { return W >= 1 && W <= 8 && m_in(M, kCritMenu, 5); }

hipError_t launch_persistent_crit(const Inst* d_insts, const int* d_order, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_persistent_crit, dim3(n), dim3(512), 0, st, d_insts, d_order, n);
  return hipGetLastError();
}

bool geometry_supported_long_batch(int W, int M) { return W >= 1 && W <= 8 && m_in(M, kLongMenu, 8); }

hipError_t launch_spans(const int32_t* path, const float* scores, int T, int blank, int max_spans,
                        int32_t* tok, int32_t* start, int32_t* end, float* score, int32_t* count,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_spans, dim3(1), dim3(1024), 0, st, path, scores, T, blank, max_spans, tok, start,
                     end, score, count);
  return hipGetLastError();
}

hipError_t launch_fill(int* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_serve(const ServeItem* d_items, ServeBox* d_box, const int32_t* d_stop,
                        uint64_t epoch, int64_t idle_limit, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_serve, dim3(grid), dim3(kWave * kServeWaves), 0, st, d_items, d_box, d_stop,
                     epoch, idle_limit);
  return hipGetLastError();
}

bool geometry_supported_serve(int W, int M) {
  return W >= 1 && W <= kServeWaves && m_in(M, kPackMenuK, 8);
}

static const int kServePartMenu[] = {4, 6, 8};
bool geometry_supported_serve_parts(int W, int M) {
  return W > 0 && W <= kServePartWaves * kServeMaxParts && W <= kXWaves * kXMaxGroups &&
         m_in(M, kServePartMenu, 3);
}

int persistent_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent, kWave * kPackWaves, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace ctca
