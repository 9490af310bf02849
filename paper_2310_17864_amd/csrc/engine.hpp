// gfx950 device engine for CTC forced alignment.
//
// The method (paper Sec. 4, "CTC-based forced alignment"; CTC formalism of
// Graves et al. 2006): Viterbi over the blank-interleaved trellis of S = 2L+1
// states,
//   a_t(s) = E[t, y'_s] + max(a_{t-1}(s), a_{t-1}(s-1), a_{t-1}(s-2) if skip(s)),
// ties resolved towards the smaller displacement, end state S-1 or S-2, then a
// backtrack to a per-frame label path.
//
// Work split: one instance runs on W wavefronts ("segments"); segment w owns
// 64*M consecutive states and lane l of it owns M consecutive states, so the
// whole a_{t-1} column lives in VGPRs and every state except the first two of
// a lane finds its predecessors in its own registers.  The one value a lane
// needs from its left neighbour (that neighbour's last state) moves by a DPP
// wave_shr:1; the value a segment needs from the previous segment moves
// through a small LDS ring guarded by counters, so segments never meet at a
// barrier: segment w may run up to a few 32-frame blocks behind segment w-1.
//
// Per frame, a blank state and the label state above it share their work:
// the blank's compare and select pick the better of the two states below the
// label (ties to the nearer one), which is also the label's best way in from
// below when it may skip, so the label adds one bitwise select (its skip
// permission), one compare and one select.  Each state then takes one float
// add and one v_addc_co_u32: the compare's lane mask is shifted straight into
// a per-lane 32-frame word, so backpointers cost one bit per state and frame
// (a label's choice between s-1 and s-2 is the blank's bit of the same frame)
// and are stored with coalesced dword stores.
//
// Emission rows reach LDS in chunks of 4 rows by direct global->LDS loads,
// one chunk ahead; label states then read their class column from a ring of
// two 4-row halves at a static offset.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "internal.hpp"

namespace ctca {

// ---- LDS structures ------------------------------------------------------

struct SegSync {
  int prod;          // boundary values published by this segment (count)
  int cons;          // previous segment's values consumed by this segment (count)
  int done;          // 1 once this segment's backpointers are stored
  int bad;           // 1 if this segment saw an invalid label
  float bnd[kBnd + 1];   // a_t(last state of this segment) in slot bslot(t)
};

// Ring slot of frame t's boundary value: 0 for t = 0, then 1 + (t-1) mod kBnd,
// so the 8 frames 8g+1 .. 8g+8 of a group sit in consecutive slots (fixed
// offsets from the group's first).
static_assert((kBnd & (kBnd - 1)) == 0 && kBnd % kUnroll == 0, "ring of whole groups");
__device__ __forceinline__ int bslot(int t) { return t == 0 ? 0 : ((t - 1) & (kBnd - 1)) + 1; }

typedef __attribute__((address_space(3))) float lds_f32;

// An LDS address held in a vector register (the compiler would otherwise
// copy it from a scalar register before every access).
__device__ __forceinline__ lds_f32* vreg_lds(const float* p) {
  uint32_t a = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void*)p;
  asm volatile("v_mov_b32 %0, %1" : "=v"(a) : "v"(a));
  return (lds_f32*)(uintptr_t)a;
}

constexpr int kSpinLimit = 1 << 26;   // bounded waits: ~seconds, never forever

__device__ __forceinline__ float neg_inf() { return -__builtin_inff(); }

// lane l receives src from lane l-1; lane 0 receives `old`.
__device__ __forceinline__ float shr1(float src, float old) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, src),
                                         0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}

// Lane masks: bit l of a 64-bit mask is lane l's predicate (a v_cmp result).
__device__ __forceinline__ uint64_t gt_mask(float x, float y) {
  return __builtin_amdgcn_ballot_w64(x > y);
}

// m ? x : y per lane, selected by an SGPR lane mask (one v_cndmask_b32).
__device__ __forceinline__ float sel(uint64_t m, float x, float y) {
  float r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(y), "v"(x), "s"(m));
  return r;
}

// acc = 2*acc + (lane's bit of m): the mask enters as the carry of one
// v_addc_co_u32, so a backpointer bit costs one VALU op and no packing.
__device__ __forceinline__ uint32_t shift_in(uint32_t acc, uint64_t m) {
  uint32_t r;   // the unused carry-out goes to VCC
  asm("v_addc_co_u32_e64 %0, vcc, %1, %1, %2" : "=v"(r) : "v"(acc), "s"(m) : "vcc");
  return r;
}

__device__ __forceinline__ int lds_load_acq(int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_store_rel(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Waits until *p >= need; returns false if the spin limit ran out.
__device__ __forceinline__ bool wait_geq(int* p, int need) {
  for (int n = 0; n < kSpinLimit; ++n) {
    if (lds_load_acq(p) >= need) return true;
    __builtin_amdgcn_s_sleep(1);
  }
  return false;
}

// ---- one frame of the recurrence for a lane's M states ---------------------
//
// a[j] holds a_{t-1} for state sbase+j on entry and a_t on exit.  Slot pairs
// (blank 2p, label 2p+1) are updated from the top down so every read sees
// a_{t-1}.  nb is a_{t-1} of the state just below this lane's first one (one
// DPP shift of the lanes' top states, lane 0 keeping the boundary value).
// With x = a(s), y = a(s-1), z = a(s-2) for label s, the strict rule picks
// s-2 iff z > y and z > x, s-1 iff y >= z and y > x, else s; the blank s-1
// has already compared z with y (its own s-1 and s), so the label compares
// x with the blank's winner only.  A label that may not skip compares with y
// alone: its permission is a per-lane all-ones / zero word kb[p] that picks
// the blank's winner or y bit by bit (v_bfi_b32, no scalar-unit round trip).

// (k & x) | (~k & y) per lane: one v_bfi_b32.
__device__ __forceinline__ float bitsel(uint32_t k, float x, float y) {
  float r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(k), "v"(x), "v"(y));
  return r;
}

// pub: lane 63 of a segment with a segment above (pub_seg, uniform) stores
// a_t of its top state to *pub as soon as the top pair is done, so the LDS
// write has the rest of the frame to complete.
template <int M>
__device__ __forceinline__ void dp_frame(float (&a)[M], uint32_t (&acc)[bp_words_per_lane(M)],
                                         const uint32_t (&kb)[M / 2], float nb, float eb,
                                         const float (&e)[M / 2], bool pub_seg, bool pub_lane,
                                         lds_f32* pub) {
#pragma unroll
  for (int p = M / 2 - 1; p >= 0; --p) {
    const int jb = 2 * p, jl = 2 * p + 1;
    const float y = a[jb];
    const float z = (jb >= 1) ? a[jb - 1] : nb;
    const uint64_t cb = gt_mask(z, y);          // blank: came from below
    const float wb = sel(cb, z, y);             // the better of z, y
    const float from_below = bitsel(kb[p], wb, y);
    const uint64_t cl = gt_mask(from_below, a[jl]);   // label: came from below
    const float wl = sel(cl, from_below, a[jl]);
    acc[plane_word(M, plane_of(M, jl))] = shift_in(acc[plane_word(M, plane_of(M, jl))], cl);
    acc[plane_word(M, plane_of(M, jb))] = shift_in(acc[plane_word(M, plane_of(M, jb))], cb);
    a[jl] = e[p] + wl;
    a[jb] = eb + wb;
    if (p == M / 2 - 1 && pub_seg) {
      if (pub_lane) *pub = a[M - 1];
    }
  }
}

// ---- emission rows: HBM -> LDS by direct loads ------------------------------
//
// The rows of frames t = 2k+1, 2k+2 form chunk k (frame 0 is read directly at
// initialisation).  A wave's ring holds four 2-row quarters; chunk k lives in
// quarter k % 4, which is static inside the unrolled 8-frame group.  HBM rows
// are 16-byte aligned with a stride of 32 or 256 floats (the host pads other
// class counts) and move with global_load_lds_dwordx4: one instruction per
// row, 16 bytes per lane, no VGPR staging.
//
// The copies are issued from inline assembly: the compiler does not see them
// as LDS writes, so it adds no waits of its own before ring reads, and the
// kernel orders them itself.  Each row copy is one vector-memory operation and
// loads complete in issue order; stores (the backpointer words) may complete
// out of order relative to loads, so no wait counts on them: waiting until at
// most N operations are outstanding, N = the number of row copies issued after
// the target, also waits out every store issued after the target.
//
// Schedule: at the end of the last frame of chunk k-1 (an odd frame of the
// group) wait for chunk k, then copy chunk k+3 into the quarter chunk k-1 has
// just vacated.  The copies of chunks k+1 and k+2 follow chunk k's, so the
// wait is vmcnt(4).
constexpr int kDmaPerChunk = 2;
constexpr int kDmaAfter = 2 * kDmaPerChunk;
typedef __attribute__((address_space(3))) void lds_void_t;

// A wave's emission ring: kRing rows of kMaxC floats in LDS.
struct Ring {
  float* base;
};

__device__ __forceinline__ float* ring_quarter(const Ring& r, int q) { return r.base + q * 2 * kMaxC; }

// One 16-byte-per-lane copy of global memory into LDS at lds_dst + 16*lane
// by the lanes in `mask`: lane l reads row + lane_off[l] (row in scalar
// registers, the per-lane byte offset in a vector register, so the address
// costs no vector instruction).  M0 holds the LDS address; one wait state
// separates its write from the copy; EXEC is restored before the block ends.
__device__ __forceinline__ void dma_row(const float* row, uint32_t lane_off, float* lds_dst, uint64_t mask) {
  const uint32_t l = (uint32_t)(uintptr_t)(lds_void_t*)lds_dst;
  uint64_t saved;
  asm volatile(
      "s_mov_b64 %0, exec\n\t"
      "s_mov_b64 exec, %4\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %2, %3\n\t"
      "s_mov_b64 exec, %0"
      : "=&s"(saved)
      : "s"(l), "v"(lane_off), "s"(row), "s"(mask)
      : "memory", "m0");
}

// 1 KB rows: 64 lanes x 16 bytes.  128-byte rows: lanes 0..7 (the others
// would only write copies into the unused part of the LDS row: 7/8 of the
// row copy's LDS bandwidth).
__device__ __forceinline__ uint32_t dma_lane_off(int lane) { return 16u * (uint32_t)lane; }
__device__ __forceinline__ uint64_t dma_mask(int hs) { return hs == kMaxC ? ~0ull : 0xFFull; }

__device__ __forceinline__ void dma_chunk(const float* em, int T, int hs, int k, uint32_t lane_off,
                                          float* quarter) {
  const uint64_t mask = dma_mask(hs);
#pragma unroll
  for (int r = 0; r < kDmaPerChunk; ++r) {
    int row = 2 * k + 1 + r;
    row = row < T ? row : T - 1;                     // clamped: always issued
    // strides are 32 or 256 floats: the byte offset is one 64-bit shift
    const int sh = hs == kMaxC ? 10 : 7;
    dma_row((const float*)((const char*)em + ((uint64_t)(uint32_t)row << sh)), lane_off, quarter + r * kMaxC,
            mask);
  }
}

__device__ __forceinline__ void wait_dma() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Waits until at most N vector-memory operations are outstanding.
template <int N>
__device__ __forceinline__ void wait_vm_keep() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// ---- boundaries between workgroups (multi layout) ---------------------------
//
// A segment whose lower neighbour runs in another workgroup copies each
// block's boundary values from the global ring into an LDS ring of its own
// (`in_lds`), after which the frame loop reads them exactly as from an LDS
// neighbour; a segment whose upper neighbour runs in another workgroup
// publishes each finished block from its own LDS ring to the global one.
struct XLink {
  XChan* in_ch = nullptr;    // ring from the lower neighbour's workgroup
  XChan* out_ch = nullptr;   // ring to the upper neighbour's workgroup
  SegSync* in_lds = nullptr; // local copy of the incoming values
  int wl = 0;                // wave index in the workgroup
  uint32_t tag = 0;          // the launch's generation tag (x_gen_tag)
};

// Polls of global memory take a round trip each: a smaller bound (~seconds).
constexpr int kXSpinLimit = 1 << 20;

__device__ __forceinline__ uint64_t x_load(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void x_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Copies boundary values i0 .. i0+cnt-1 (cnt <= 64) from the global ring to
// dst, waiting (bounded) until every slot holds this launch's tag and its
// index.  Then tells the producer which values it may overwrite: those below
// i0+cnt-1, since the next pull starts with that last value again (a
// block's pull includes the first value of the next block).
__device__ __forceinline__ bool x_pull(XChan* ch, SegSync* dst, int i0, int cnt, int lane, uint32_t tag) {
  const int i = i0 + lane;
  for (int it = 0; it < kXSpinLimit; ++it) {
    uint64_t v = 0;
    if (lane < cnt) v = x_load(&ch->slot[i % kXRing]);
    const bool ok = lane >= cnt || (uint32_t)(v >> 32) == (tag | (uint32_t)i);
    if (__builtin_amdgcn_ballot_w64(!ok) == 0) {
      if (lane < cnt) dst->bnd[bslot(i)] = __builtin_bit_cast(float, (uint32_t)v);
      if (lane == 0)
        __hip_atomic_store(&ch->cons, (int32_t)(tag | (uint32_t)(i0 + cnt - 1)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
      return true;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

// Waits (bounded) until the consumer has released every value that slot
// reuse up to index i_end (exclusive) would overwrite (those below
// i_end - kXRing).  `seen` caches its progress; a count left by another
// launch (other tag) counts as none.
__device__ __forceinline__ bool x_room(XChan* ch, int i_end, int& seen, uint32_t tag) {
  for (int it = 0; it < kXSpinLimit && i_end - kXRing > seen; ++it) {
    const uint32_t c = (uint32_t)__hip_atomic_load(&ch->cons, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if ((c & ~kXIdxMask) == tag) seen = (int)(c & kXIdxMask);
    if (i_end - kXRing > seen) __builtin_amdgcn_s_sleep(2);
  }
  return i_end - kXRing <= seen;
}

// Publishes boundary values i0 .. i0+cnt-1 (cnt <= 64) of src to the ring.
__device__ __forceinline__ void x_push(XChan* ch, const SegSync* src, int i0, int cnt, int lane, uint32_t tag) {
  if (lane < cnt) {
    const int i = i0 + lane;
    const uint32_t bits = __builtin_bit_cast(uint32_t, src->bnd[bslot(i)]);
    x_store(&ch->slot[i % kXRing], ((uint64_t)(tag | (uint32_t)i) << 32) | bits);
  }
}

// Where segment outcomes go for the backtrack.
struct FwdOut {
  float total;
  int send;
  int ok;   // 0 = a wait ran out (device watchdog)
};

// ---- forward pass of one segment -----------------------------------------
//
// `sy` points at the SegSync of segment 0 of this instance; the caller has
// cleared it and passed a workgroup barrier after `prologue_check`.
// kX: multi layout; `sy` is then this workgroup's SegSync array and xl says
// which neighbours sit in other workgroups.
//
// kMode (checkpointed long form, CkArgs): kModeCkFirst keeps the column of
// every ck->every-th frame and stores no backpointers; kModeCkSeg starts from
// column ck->col instead of frame 0 and has no end state of its own.
template <int M, bool kX = false, int kMode = kModeFull>
__device__ __forceinline__ FwdOut segment_forward(const Inst& in, const int w, const int lane,
                                                  const Ring& ring, SegSync* sy, bool labels_bad,
                                                  const XLink& xl = XLink{},
                                                  const CkArgs* ck = nullptr) {
  const int T = in.T, L = in.L, blank = in.blank, W = in.W;
  const int S = 2 * L + 1;                  // state counts fit int32 (host-checked)
  const int sbase = (w * kWave + lane) * M;
  const float* em = in.em;
  FwdOut out{neg_inf(), 0, 1};
  if (labels_bad) return out;

  // a1: per-state metadata.  Label states read their class column from the
  // ring at byte offset 4*label; padding states (s >= S) read the blank
  // column and can neither skip nor feed a real state.
  int eoff[M / 2];
  uint32_t skip[M / 2];   // all ones: may enter from two states below, 0: may not
#pragma unroll
  for (int jj = 0; jj < M / 2; ++jj) {
    const int s = sbase + 2 * jj + 1;
    int lab = blank;
    bool sk = false;
    if (s < S) {
      lab = in.lab[(s - 1) / 2];
      if (s >= 3) sk = lab != in.lab[(s - 3) / 2];
    }
    eoff[jj] = lab;
    skip[jj] = sk ? ~0u : 0u;
  }

  // a3: frame 0.  Only states 0 and 1 start finite.  (A checkpointed
  // stretch starts from its stored column instead.)
  float a[M];
  if constexpr (kMode == kModeCkSeg) {
    const float* col = ck->ck + (int64_t)ck->col * ck->spad + sbase;
#pragma unroll
    for (int j = 0; j < M; ++j) a[j] = col[j];
  } else {
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int s = sbase + j;
      a[j] = neg_inf();
      if (s == 0) a[j] = em[blank];
      if (s == 1 && S > 1) a[j] = em[in.lab[0]];
    }
  }
  if constexpr (kMode == kModeCkFirst) {
    float* col = ck->ck + sbase;   // column 0
#pragma unroll
    for (int j = 0; j < M; ++j) col[j] = a[j];
  }

  const bool has_next = w + 1 < W, has_prev = w > 0;
  const int wl = kX ? xl.wl : w;          // index into sy
  // neighbours in other workgroups (multi layout only)
  const bool prev_x = kX && has_prev && xl.in_ch != nullptr;
  const bool next_x = kX && has_next && xl.out_ch != nullptr;
  SegSync* me = sy + wl;
  SegSync* prev = has_prev ? (prev_x ? xl.in_lds : sy + wl - 1) : nullptr;
  SegSync* next = (has_next && !next_x) ? sy + wl + 1 : nullptr;
  // Boundary values are read every frame through a pointer that always points
  // into the SegSync array (the compiler then knows it cannot alias the ring).
  // The lowest segment reads -inf (the state below state 0) from a ring no
  // other segment of the instance uses: the top segment's own (a top segment
  // never publishes) or, in the multi layout, the first workgroup's copy of
  // incoming values (it has none).
  SegSync* pv = prev;
  if (!has_prev) {
    pv = kX ? xl.in_lds : sy + (W - 1);
    for (int k = lane; k <= kBnd; k += kWave) pv->bnd[k] = neg_inf();
  }
  int x_seen = 0;                         // consumer progress seen by a cross-workgroup producer
  if (has_next) {
    if (lane == kWave - 1) me->bnd[0] = a[M - 1];
    if (next_x)
      x_push(xl.out_ch, me, 0, 1, lane, xl.tag);
    else
      lds_store_rel(&me->prod, 1);
  }

  const int nsteps = T - 1;               // frames 1..T-1
  const int nblk = (nsteps + kBlk - 1) / kBlk;
  constexpr int NQ = bp_words_per_lane(M);
  const int ngrp = (int)bp_groups(T);
  uint32_t* bpw = in.bp + (int64_t)w * ngrp * NQ * kWave + lane;

  const int hs = in.stride;
  const uint32_t dma_off = dma_lane_off(lane);
  // Small lanes read each frame's emissions one frame ahead (M/2+1 more
  // registers), hiding the LDS latency behind the previous frame's work.
  constexpr bool kAhead = M <= 16;
  float eb_c = 0.f, e_c[M / 2];
#pragma unroll
  for (int jj = 0; jj < M / 2; ++jj) e_c[jj] = 0.f;
  if (nsteps > 0) {
    dma_chunk(em, T, hs, 0, dma_off, ring_quarter(ring, 0));
    dma_chunk(em, T, hs, 1, dma_off, ring_quarter(ring, 1));
    dma_chunk(em, T, hs, 2, dma_off, ring_quarter(ring, 2));
    wait_vm_keep<kDmaAfter>();     // chunk 0 has landed
    dma_chunk(em, T, hs, 3, dma_off, ring_quarter(ring, 3));
    if constexpr (kAhead) {
      const float* r0 = ring_quarter(ring, 0);
      eb_c = r0[blank];
#pragma unroll
      for (int jj = 0; jj < M / 2; ++jj) e_c[jj] = r0[eoff[jj]];
    }
  }

  uint32_t acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0;
  lds_f32* const ebp = vreg_lds(ring.base + blank);   // the blank column of ring row 0

  // neighbours in one workgroup hand over boundary values every 8-frame
  // group in the batched and single kernels, every 32-frame block in the
  // multi-workgroup layout (its frames are short: few states per lane)
  constexpr bool kGroupFlow = !kX;
  bool alive = true;
  int u = 0;
  for (int b = 0; b < nblk && alive; ++b) {
    const int n = (nsteps - 32 * b) < kBlk ? (nsteps - 32 * b) : kBlk;
    // flow control with a neighbour in another workgroup: once per 32-frame
    // block (one value past the block: the last frame reads the next one
    // ahead)
    if (prev_x) alive &= x_pull(xl.in_ch, prev, 32 * b, n + 1, lane, xl.tag);   // values 32b .. 32b+n
    if (next_x) alive &= x_room(xl.out_ch, 32 * b + n + 1, x_seen, xl.tag);
    if constexpr (!kGroupFlow) {
      if (has_prev && !prev_x) alive &= wait_geq(&prev->prod, 32 * b + n + 1);
      if (has_next && !next_x && 32 * b + n - kBnd + 1 > 0)
        alive &= wait_geq(&next->cons, 32 * b + n - kBnd + 1);
    }
    if (!alive) break;
    float bv_c = 0.f;

#pragma unroll 1
    for (int g = 0; g < kBlk / kUnroll; ++g) {
      const int ng = n - kUnroll * g;            // frames of this group (may be < 8 or <= 0)
      if (ng <= 0) break;
      const int ubase = 32 * b + kUnroll * g;
      const int ne = ng < kUnroll ? ng : kUnroll;
      // flow control inside the workgroup, once per 8-frame group (one value
      // past the group, read ahead by its last frame): a segment trails the
      // one below by about a group, so the emission rows it reads again are
      // still in the L2 the lower segment brought them into
      if constexpr (kGroupFlow) {
        if (has_prev && !prev_x) alive &= wait_geq(&prev->prod, ubase + ne + 1);
        if (has_next && !next_x && ubase + ne - kFlowWin + 1 > 0)
          alive &= wait_geq(&next->cons, ubase + ne - kFlowWin + 1);
        if (!alive) break;
      }
      if (g == 0) bv_c = pv->bnd[bslot(32 * b)];   // boundary value of the block's first frame
      // this group's boundary slots: frame ubase+i+1 at offset i
      lds_f32* const grp_rd = vreg_lds(pv->bnd + bslot(ubase + 1));
      lds_f32* const grp_wr = vreg_lds(me->bnd + bslot(ubase + 1));
      // One frame: i is the frame's static position in the group.
      auto frame = [&](auto ic) __attribute__((always_inline)) {
        constexpr int i = decltype(ic)::value;
        const int uu = ubase + i;                // computes frame t = uu + 1
        if constexpr (!kAhead) {
          const float* rc = ring_quarter(ring, (i / 2) % 4) + (i % 2) * kMaxC;
          eb_c = rc[blank];
#pragma unroll
          for (int jj = 0; jj < M / 2; ++jj) e_c[jj] = rc[eoff[jj]];
        }
        if constexpr (i % 2 == 1) {
          // a2: wait for chunk k (the next frame's) and refill chunk k-1's
          // quarter with chunk k+3 once its reads have completed (with
          // read-ahead, this frame's values were read during the last one)
          const int k = (uu + 1) / 2;
          wait_vm_keep<kDmaAfter>();
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
          dma_chunk(em, T, hs, k + 3, dma_off, ring_quarter(ring, (i / 2) % 4));
        }
        // this frame's boundary value was read one frame ahead: lane 0 takes
        // it, the other lanes their left neighbour's top state.  Done before
        // the next frame's reads are issued (the compiler waits for every
        // outstanding LDS read at this use), then the reads, then this frame's
        // arithmetic, which hides their latency.
        const float nb = shr1(a[M - 1], bv_c);
        __builtin_amdgcn_sched_barrier(0);
        bv_c = grp_rd[i];
        float eb_n = 0.f, e_n[M / 2];
        if constexpr (kAhead) {
          // the next frame's values, read while this frame computes
          const float* rn = ring_quarter(ring, ((i + 1) / 2) % 4) + ((i + 1) % 2) * kMaxC;
          eb_n = ebp[(((i + 1) / 2) % 4) * 2 * kMaxC + ((i + 1) % 2) * kMaxC];
#pragma unroll
          for (int jj = 0; jj < M / 2; ++jj) e_n[jj] = rn[eoff[jj]];
        }
        __builtin_amdgcn_sched_barrier(0);
        dp_frame<M>(a, acc, skip, nb, eb_c, e_c, has_next, lane == kWave - 1, grp_wr + i);
        if constexpr (kAhead) {
          eb_c = eb_n;
#pragma unroll
          for (int jj = 0; jj < M / 2; ++jj) e_c[jj] = e_n[jj];
        }
        u = uu;
        // keep each frame's instructions together: bounds live registers
        __builtin_amdgcn_sched_barrier(0);
      };
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, 1>;
      using I2 = std::integral_constant<int, 2>;
      using I3 = std::integral_constant<int, 3>;
      using I4 = std::integral_constant<int, 4>;
      using I5 = std::integral_constant<int, 5>;
      using I6 = std::integral_constant<int, 6>;
      using I7 = std::integral_constant<int, 7>;
      if (ng >= kUnroll) {
        // full group: straight-line code
        frame(I0{}); frame(I1{}); frame(I2{}); frame(I3{});
        frame(I4{}); frame(I5{}); frame(I6{}); frame(I7{});
      } else {
        // The utterance's last, short group (< 8 frames): the copies issued
        // so far already cover it (they run 6 frames ahead), so wait for them
        // all and read the ring directly, one frame per iteration.
        wait_dma();
#pragma unroll 1
        for (int i = 0; i < ng; ++i) {
          const int uu = ubase + i;
          const float* rc = ring_quarter(ring, (i >> 1) & 3) + (i & 1) * kMaxC;
          const float eb = rc[blank];
          float e[M / 2];
#pragma unroll
          for (int jj = 0; jj < M / 2; ++jj) e[jj] = rc[eoff[jj]];
          dp_frame<M>(a, acc, skip, shr1(a[M - 1], pv->bnd[bslot(uu)]), eb, e, has_next,
                      lane == kWave - 1, grp_wr + i);
          u = uu;
        }
      }
      // a5: flush the group's backpointer words; frame i of plane r of word q
      // lands at bit 31 - (R*i + r) (left-aligned when the group is short)
      if constexpr (kMode != kModeCkFirst) {
        const int gi = 4 * b + g;
        uint32_t* dst = bpw + (int64_t)gi * NQ * kWave;
        const int nf = ng < kUnroll ? ng : kUnroll;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int sh = 32 - planes_in_word(M, q) * nf;
          dst[q * kWave] = acc[q] << sh;
        }
      }
      if constexpr (kGroupFlow) {
        if (has_next && !next_x) lds_store_rel(&me->prod, ubase + ne + 1);
        if (has_prev && !prev_x) lds_store_rel(&me->cons, ubase + ne);
      }
    }

    if constexpr (kMode == kModeCkFirst) {
      // the column of frame 32b+32 when it starts a later stretch (every
      // stretch start below T-1 ends a whole block)
      const int tl = 32 * b + n;
      if (n == kBlk && tl % ck->every == 0 && tl < T - 1) {
        float* col = ck->ck + (int64_t)(tl / ck->every) * ck->spad + sbase;
#pragma unroll
        for (int j = 0; j < M; ++j) col[j] = a[j];
      }
    }
    if (next_x && alive) x_push(xl.out_ch, me, 32 * b + 1, n, lane, xl.tag);   // values 32b+1 .. 32b+n
    if constexpr (!kGroupFlow) {
      if (has_next && !next_x) lds_store_rel(&me->prod, 32 * b + n + 1);
      if (has_prev && !prev_x) lds_store_rel(&me->cons, 32 * b + n);
    }
  }
  out.ok = alive ? 1 : 0;
  wait_dma();   // no copy into LDS may outlive this instance

  // a6: end state, in the segment that holds S-1 and S-2
  if (w == W - 1 && kMode != kModeCkSeg) {
    float v1 = neg_inf(), v2 = neg_inf();
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int s = sbase + j;
      if (s == S - 1) v1 = a[j];
      if (s == S - 2) v2 = a[j];
    }
    const int q1 = (S - 1) - w * kWave * M;
    const int l1 = q1 / M;
    const float f1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v1), l1));
    if (S == 1) {
      out.total = f1;
      out.send = 0;
    } else if (q1 == 0) {
      // S-1 opens this segment (layouts whose top segment holds one state):
      // S-2 is the last state of the segment below, and its value at the
      // last frame is the final entry of the boundary ring, which the last
      // block already waited for (with one frame there is no ring entry, and
      // a_0(S-2) = -inf since S-2 >= 2)
      float f2 = neg_inf();
      if (prev_x) out.ok = 0;   // not a layout of the multi-workgroup kernel
      else if (in.T > 1) f2 = pv->bnd[bslot(in.T - 1)];
      const bool take2 = f2 > f1;
      out.total = take2 ? f2 : f1;
      out.send = take2 ? S - 2 : S - 1;
    } else {
      const int q2 = q1 - 1;
      const int l2 = q2 / M;
      const float f2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v2), l2));
      const bool take2 = f2 > f1;
      out.total = take2 ? f2 : f1;
      out.send = take2 ? S - 2 : S - 1;
    }
  }
  return out;
}

// ---- a1 prologue: validate labels ------------------------------------------
// Every segment checks the labels of its own states; the instance's verdict is
// the OR over segments after a workgroup barrier.
template <int M>
__device__ __forceinline__ bool prologue_check(const Inst& in, int w, int lane) {
  const int S = 2 * in.L + 1;
  const int sbase = (w * kWave + lane) * M;
  bool bad = false;
#pragma unroll
  for (int jj = 0; jj < M / 2; ++jj) {
    const int s = sbase + 2 * jj + 1;
    if (s < S) {
      const int v = in.lab[(s - 1) / 2];
      bad |= (v < 0) | (v >= in.C) | (v == in.blank);
    }
  }
  return __builtin_amdgcn_ballot_w64(bad) != 0;
}

// ---- a7: backtrack ---------------------------------------------------------
//
// The chase s_{t-1} = s_t - k_t(s_t) runs in scalar registers, 32 frames per
// block.  Over one block the state drops by at most 62, so the block's codes
// for the 63 states at and below the block's top state sit one per lane (the
// "band"), as 2-bit codes built from each state's own 32 frame bits and, for
// a label state that may skip, those of the blank state below it (the next
// lane: which of the two states below the label it came from); a frame then
// costs one readlane.  Lane i records the state of the block's
// frame i; its label is fetched after the chase and stored one block later.
//
// Fetches run two blocks ahead: at the top of block b (state e_b) the raw
// words of block b-2 are requested for the 192 states below e_b (three
// 64-state windows; the top of block b-2 is at most 124 below e_b), with the
// two labels that decide each label state's skip permission.  After block
// b-1's chase has fixed that top, the windows are realigned to it with
// ds_bpermute and only the 64-state band is unpacked.  Every fetch is issued
// unconditionally (clamped addresses; masking happens at unpack time, since
// overwriting a register with a load in flight would wait for it), so the
// compiler's vmcnt waits count exactly; the path stores go out through
// inline assembly: the compiler does not see them, which keeps its waits for
// loads exact instead of draining all memory operations (loads complete in
// issue order among themselves whatever the stores do).

// A state's codes k for the 32 frames of a block, 2 bits per frame: frame i
// of the block at bits 31-2i, 30-2i of c0 (i < 16) or 63-2i, 62-2i of c1.
struct Band {
  uint32_t c0, c1;
};

// bit j of the low 16 bits -> bit 2j
__device__ __forceinline__ uint32_t spread16(uint32_t x) {
  x &= 0xFFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// codes from the "came from below" and "came from two below" words (frame i
// at bit 31-i): k = 2 where the second is set, else the first bit
__device__ __forceinline__ Band make_band(uint32_t mv, uint32_t sk) {
  const uint32_t lo = mv & ~sk;
  return Band{(spread16(sk >> 16) << 1) | spread16(lo >> 16), (spread16(sk) << 1) | spread16(lo)};
}

// Raw backpointer words of one state for the 4 groups of a block (the word
// holding its plane), plus the two labels whose difference is a label
// state's skip permission (label 0 twice for other states).  The bit of the
// blank below a label state is the next band lane's own bit.
struct RawWin {
  uint32_t wm[4];
  int32_t la, lb;
};

// Where state q's plane sits in a lane's words.
struct PlaneLoc {
  int wseg, ln;          // segment, lane
  int qm, pm, rm;        // word, bit offset, planes in the word
  bool odd;
};

template <int M>
__device__ __forceinline__ PlaneLoc plane_loc(int q) {
  PlaneLoc p;
  const int segsz = kWave * M;
  p.wseg = q / segsz;
  const int rr = q - p.wseg * segsz;
  p.ln = rr / M;
  const int j = rr - p.ln * M;
  p.odd = j % 2;
  const int pown = plane_of(M, j);
  p.qm = plane_word(M, pown);
  p.pm = plane_pos(M, pown);
  p.rm = planes_in_word(M, p.qm);
  return p;
}

typedef __attribute__((address_space(1))) const uint32_t gu32_t;
typedef __attribute__((address_space(1))) const int32_t gi32_t;

// labp: the labels (any readable int32 array when there are none: only
// state 0 then exists and reads index 0).  Groups are read at fixed offsets
// from the block's first (the layout holds whole blocks).
template <int M>
__device__ __forceinline__ RawWin load_win(const Inst& in, const int* labp, int blk, int ngrp, int q) {
  RawWin r;
  constexpr int NQ = bp_words_per_lane(M);
  const PlaneLoc p = plane_loc<M>(q > 0 ? q : 0);
  gu32_t* base = (gu32_t*)in.bp + ((int64_t)p.wseg * ngrp + 4 * blk) * NQ * kWave + p.qm * kWave + p.ln;
#pragma unroll
  for (int g = 0; g < 4; ++g) r.wm[g] = base[g * NQ * kWave];
  const bool lab2 = (q >= 3) && (q % 2);          // a label state with a label two below
  r.la = ((gi32_t*)labp)[lab2 ? (q - 1) / 2 : 0];
  r.lb = ((gi32_t*)labp)[lab2 ? (q - 3) / 2 : 0];
  return r;
}

// The 8 frame bits of plane offset p in a word of R interleaved planes
// (frame i at bit 31-(R*i+p)), moved to the top byte in frame order (frame i
// at bit 31-i): mask, then merge neighbours in three doubling steps.
__device__ __forceinline__ uint32_t gather8(uint32_t w, int R, int p) {
  const uint32_t m0 = R == 4 ? 0x88888888u : R == 3 ? 0x92492400u : R == 2 ? 0xAAAA0000u : 0xFF000000u;
  const uint32_t m1 = R == 4 ? 0xC0C0C0C0u : R == 3 ? 0xC30C3000u : R == 2 ? 0xCCCC0000u : 0xFF000000u;
  const uint32_t m2 = R == 4 ? 0xF000F000u : R == 3 ? 0xF00F0000u : R == 2 ? 0xF0F00000u : 0xFF000000u;
  uint32_t x = (w << p) & m0;
  x = (x | (x << (R - 1))) & m1;
  x = (x | (x << (2 * R - 2))) & m2;
  x = (x | (x << (4 * R - 4))) & 0xFF000000u;
  return x;
}

__device__ __forceinline__ uint32_t bperm(uint32_t v, int src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane * 4, (int)v);
}

// lane l receives src from lane l+1 (lane 63 keeps src).
__device__ __forceinline__ uint32_t shl1(uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)src, (int)src, 0x130 /* wave_shl:1 */, 0xf, 0xf, false);
}

// Band of state q (lane l of a band of consecutive states, q = top - l) from
// its own 32 frame bits mv and the two labels fetched for it: a label state
// came from s-2 where it came from below, may skip, and the blank below it
// (the next lane) came from below too.
template <int M>
__device__ __forceinline__ Band band_from(uint32_t mv, int32_t la, int32_t lb, int q, const PlaneLoc& p) {
  if (q < 0) mv = 0u;
  const uint32_t pb = shl1(mv);
  const bool may_skip = q >= 3 && p.odd && la != lb;
  const uint32_t sk = may_skip ? (mv & pb) : 0u;
  return make_band(mv, sk);
}

// Band of state q (= the windows' top - d - lane) from three windows: realign
// with ds_bpermute and unpack, group by group.
template <int M>
__device__ __forceinline__ Band band_of(const RawWin& a, const RawWin& b, const RawWin& c, int d, int q,
                                        int lane) {
  const int x = d + lane;            // 0..191
  const int k = x >> 6, src = x & (kWave - 1);
  auto pick = [&](uint32_t va, uint32_t vb, uint32_t vc) __attribute__((always_inline)) {
    const uint32_t ra = bperm(va, src), rb = bperm(vb, src), rc = bperm(vc, src);
    return k == 0 ? ra : (k == 1 ? rb : rc);
  };
  const PlaneLoc p = plane_loc<M>(q > 0 ? q : 0);
  uint32_t mv = 0u;
#pragma unroll
  for (int g = 0; g < 4; ++g) mv |= gather8(pick(a.wm[g], b.wm[g], c.wm[g]), p.rm, p.pm) >> (kUnroll * g);
  // only whether the two labels differ matters
  const uint32_t dl = pick((uint32_t)(a.la ^ a.lb), (uint32_t)(b.la ^ b.lb), (uint32_t)(c.la ^ c.lb));
  return band_from<M>(mv, (int32_t)dl, 0, q, p);
}

// Band of state q straight from one window (no realignment).
template <int M>
__device__ __forceinline__ Band band_direct(const RawWin& a, int q) {
  const PlaneLoc p = plane_loc<M>(q > 0 ? q : 0);
  uint32_t mv = 0u;
#pragma unroll
  for (int g = 0; g < 4; ++g) mv |= gather8(a.wm[g], p.rm, p.pm) >> (kUnroll * g);
  return band_from<M>(mv, a.la, a.lb, q, p);
}

// Two frames per lookup.  In a band word, frame pair j (frames 2j+1, 2j)
// is the nibble at bits 31-4j .. 28-4j: frame 2j+1's code below, frame 2j's
// above.  The chase meets frame 2j+1 first, at the lane's own state, and
// frame 2j at the state k1 = code(2j+1) lanes further; so the upper half of
// each nibble is replaced by that lane's code (k1 <= 2: the lane itself, its
// next or the one after, moved by two DPP shifts).  One readlane then yields
// both drops.  Lanes 62 and 63 receive garbage from beyond the band; a chase
// never reaches them before the block's last pair is read.
__device__ __forceinline__ uint32_t pair_codes(uint32_t w) {
  const uint32_t n1 = shl1(w), n2 = shl1(n1);
  const uint32_t lo1 = w & 0x11111111u;          // k1 == 1
  const uint32_t lo2 = (w >> 1) & 0x11111111u;   // k1 == 2
  const uint32_t m1 = lo1 * 12u, m2 = lo2 * 12u; // the nibble's upper two bits
  const uint32_t t = (m1 & n1) | (~m1 & w);
  return (m2 & n2) | (~m2 & t);
}

// f(integral_constant<N-1>), ..., f(integral_constant<0>)
template <int N, typename F>
__device__ __forceinline__ void unroll_down(F&& f) {
  if constexpr (N > 0) {
    f(std::integral_constant<int, N - 1>{});
    unroll_down<N - 1>(f);
  }
}

// Stores the compiler does not track (see above).
__device__ __forceinline__ void store_untracked(void* p, uint32_t v) {
  asm volatile("global_store_dword %0, %1, off" ::"v"(p), "v"(v) : "memory");
}

__device__ __forceinline__ void fill_outputs(const Inst& in, int lane, int path_val, float score_val) {
  for (int t = lane; t < in.T; t += kWave) {
    in.path[t] = path_val;
    in.scores[t] = score_val;
  }
}

// out_state (nullable): receives the state of frame 0 (the checkpointed
// long form starts the previous stretch's backtrack there).
template <int M>
__device__ __forceinline__ void backtrack(const Inst& in, const FwdOut& fo, int status_in, int lane,
                                          int32_t* out_state = nullptr) {
  const int T = in.T, RS = in.stride, blank = in.blank;   // RS: emission row stride
  const float* em = in.em;
  int status = status_in;
  float total = fo.total;
  if (status == kOk && !fo.ok) status = kEdevice;
  if (status == kOk && total == neg_inf()) status = kEinfeasible;
  // start with no memory operation in flight (see the loop head below)
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)

  if (status != kOk) {
    const float fillv = (status == kEinfeasible) ? neg_inf() : __builtin_nanf("");
    fill_outputs(in, lane, -1, fillv);
    if (status != kEinfeasible) total = __builtin_nanf("");
  } else {
    const int nblk = (T - 1 + kBlk - 1) / kBlk;
    const int ngrp = (int)bp_groups(T);
    // with no labels every state is blank: the label reads hit path[0]
    const int* labp = (in.L > 0 && in.lab) ? in.lab : in.path;
    int e = fo.send;                       // state at the top of the current block
    Band cur{0u, 0u};
    // Two window sets alternate between "fetched for the block after next"
    // and "being realigned for the next block"; the loop is unrolled by two so
    // that no set is ever copied (a copy would wait for its loads).
    RawWin setA[3], setB[3];
    int ntop = e;                          // top the next block's windows were fetched below
    if (nblk > 0) {
      cur = band_direct<M>(load_win<M>(in, labp, nblk - 1, ngrp, e - lane), e - lane);
      const int nb = nblk - 2 >= 0 ? nblk - 2 : 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) setA[k] = load_win<M>(in, labp, nb, ngrp, e - k * kWave - lane);
      // enter the loop with no load in flight: the compiler's waits at the
      // loop head then only see the loop's own (exactly counted) fetches
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    }
    int pend_lab = 0, pend_odd = 0;
    int pend_t0 = -1;
    int pend_n = 0;
    // One block: fetch block b-2's windows into `fetch`, chase block b, store
    // the previous block's path, fetch this block's labels, then build block
    // b-1's band from `next`.
    auto step = [&](int b, RawWin (&next)[3], RawWin (&fetch)[3]) __attribute__((always_inline)) {
      const int n = (T - 1 - 32 * b) < kBlk ? (T - 1 - 32 * b) : kBlk;
      const int top = e;
      const int fb = b - 2 >= 0 ? b - 2 : 0;   // for b < 2 the fetch is unused
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        fetch[k] = load_win<M>(in, labp, fb, ngrp, top - k * kWave - lane);
        __builtin_amdgcn_sched_barrier(0);     // bounds live address registers
      }
      // chase frames t = 32b+n .. 32b+1: one readlane of the state's code
      // word per frame (fully unrolled for whole blocks)
      int outst = 0;                       // lane i: the state at the block's frame i
      auto step_code = [&](int i) __attribute__((always_inline)) {
        const int l = top - e;
        const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)(i < 16 ? cur.c0 : cur.c1), l);
        e -= (int)((w >> ((i < 16 ? 30 : 62) - 2 * i)) & 3u);
      };
      if (n == kBlk) {
        // whole block, two frames per readlane (pair_codes); frame i's state
        // goes to lane i by v_writelane with an immediate lane index (no
        // per-frame lane mask)
        const uint32_t w0 = pair_codes(cur.c0), w1 = pair_codes(cur.c1);
        auto chase_p = [&](auto jc) __attribute__((always_inline)) {
          constexpr int j = decltype(jc)::value;   // frames 2j+1, 2j
          constexpr int sh = 28 - 4 * (j & 7);
          asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(outst) : "s"(__builtin_amdgcn_readfirstlane(e)), "n"(2 * j + 1));
          const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)(j >= 8 ? w1 : w0), top - e);
          const int e1 = e - (int)((w >> sh) & 3u);
          asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(outst) : "s"(__builtin_amdgcn_readfirstlane(e1)), "n"(2 * j));
          e = e1 - (int)((w >> (sh + 2)) & 3u);
        };
        unroll_down<kBlk / 2>(chase_p);
      } else {
        for (int i = n - 1; i >= 0; --i) {
          outst = (lane == i) ? e : outst;
          step_code(i);
        }
      }
      // path of the previous block (its label reads have had a block's time)
      if (pend_t0 >= 0 && lane < pend_n)
        store_untracked(in.path + pend_t0 + lane, (uint32_t)(pend_odd ? pend_lab : blank));
      pend_t0 = 32 * b + 1;
      pend_n = n;
      pend_odd = outst % 2;
      pend_lab = labp[pend_odd ? (outst - 1) / 2 : 0];
      if (b > 0) {
        cur = band_of<M>(next[0], next[1], next[2], ntop - e, e - lane, lane);
        ntop = top;
      }
    };
    // both steps unconditional inside the loop (a path around the second one
    // would leave set B in flight at the loop head and force a full wait there)
    int b = nblk - 1;
    for (; b >= 1; b -= 2) {
      step(b, setA, setB);
      step(b - 1, setB, setA);
    }
    if (b == 0) step(0, setA, setB);
    if (pend_t0 >= 0 && lane < pend_n)
      store_untracked(in.path + pend_t0 + lane, (uint32_t)(pend_odd ? pend_lab : blank));
    // frame 0
    if (lane == 0) {
      const int lab0 = (e % 2 == 0) ? blank : in.lab[(e - 1) / 2];
      store_untracked(in.path, (uint32_t)lab0);
      if (out_state) store_untracked(out_state, (uint32_t)e);
    }
    // per-frame scores: emission[t, path[t]], four independent gathers per
    // lane in flight (the path stores above are complete after the wait)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    for (int t0 = 0; t0 < T; t0 += 4 * kWave) {
      int c[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = t0 + r * kWave + lane;
        c[r] = t < T ? in.path[t] : -1;
      }
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = t0 + r * kWave + lane;
        v[r] = c[r] >= 0 ? em[(int64_t)t * RS + c[r]] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = t0 + r * kWave + lane;
        if (c[r] >= 0) in.scores[t] = v[r];
      }
    }
  }
  if (lane == 0) {
    if (in.total) *in.total = total;
    if (in.status) *in.status = status;
  }
  if (in.notify) {
    // every store of this wave (path, scores, total, status) complete and
    // written back past the L2 before the flag reaches the host
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    if (lane == 0) __hip_atomic_store(in.notify, status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace ctca
