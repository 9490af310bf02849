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
// Per frame and state the work is one compare + one select for a blank state
// and two compares + two selects for a label state, one float add each, plus
// one v_addc_co_u32 per backpointer bit: the compare's lane mask is shifted
// straight into a per-lane 32-frame word ("moved one state" plane for every
// state, "skipped a state" plane for label states), so backpointers cost 1.5
// bits per state and frame and are stored with coalesced dword stores.
//
// Emission rows reach LDS in chunks of 4 rows through registers, one chunk
// ahead, with an L2 warm-up load three chunks ahead; label states then read
// their class column from a ring of 8 rows at a static offset.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace ctca {

// ---- LDS structures ------------------------------------------------------

struct SegSync {
  int prod;          // boundary values published by this segment (count)
  int cons;          // previous segment's values consumed by this segment (count)
  int done;          // 1 once this segment's backpointers are stored
  int bad;           // 1 if this segment saw an invalid label
  float bnd[kBnd];   // a_t(last state of this segment), slot t % kBnd
};

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
  uint32_t r;
  uint64_t co;
  asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(r), "=s"(co) : "v"(acc), "s"(m));
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
// a[j] holds a_{t-1} for state sbase+j on entry and a_t on exit.  States are
// updated from the top down so every read sees a_{t-1}.  nb is a_{t-1} of the
// state just below this lane's first one.  Even slots are blank states.
template <int M>
__device__ __forceinline__ void dp_frame(float (&a)[M], uint32_t (&mv)[M], uint32_t (&sk)[M / 2],
                                         const uint64_t (&skip)[M / 2], float nb, float eb,
                                         const float (&e)[M / 2]) {
#pragma unroll
  for (int j = M - 1; j >= 0; --j) {
    const float p1 = (j >= 1) ? a[j - 1] : nb;
    if (j % 2 == 0) {
      const uint64_t c1 = gt_mask(p1, a[j]);
      const float best = sel(c1, p1, a[j]);
      mv[j] = shift_in(mv[j], c1);
      a[j] = eb + best;
    } else {
      const float p2 = (j >= 2) ? a[j - 2] : nb;
      const uint64_t c1 = gt_mask(p1, a[j]);
      const float b1 = sel(c1, p1, a[j]);
      const uint64_t c2 = gt_mask(p2, b1) & skip[j / 2];
      const float b2 = sel(c2, p2, b1);
      mv[j] = shift_in(mv[j], c1);
      sk[j / 2] = shift_in(sk[j / 2], c2);
      a[j] = e[j / 2] + b2;
    }
  }
}

// ---- emission chunks: global -> registers -> LDS ring ----------------------
//
// Chunk k holds the rows of frames t = 4k+1 .. 4k+4 (frame 0 is read
// directly at initialisation) and lands in ring rows (4k) % 8 .. +3.  The
// rows are contiguous in HBM (row stride C == STRIDE, 16-byte aligned; the
// host pads other class counts beforehand), so a chunk is one contiguous
// copy of 4*STRIDE floats: 2 per lane for STRIDE 32, 16 for STRIDE 256.
template <int STRIDE>
struct Stager {
  static constexpr int kPer = kChunk * STRIDE / kWave;
  static constexpr int kVec = kPer >= 4 ? 4 : kPer;      // floats per load
  float v[kPer];

  __device__ __forceinline__ void load(const float* em, int T, int k, int lane) {
    const int row0 = 4 * k + 1;
    if (row0 >= T) return;
    const float* src = em + (int64_t)row0 * STRIDE;
    const int lim = ((T - row0) < kChunk ? (T - row0) : kChunk) * STRIDE;
#pragma unroll
    for (int q = 0; q < kPer / kVec; ++q) {
      const int e = kVec * (lane + kWave * q);
      if (e < lim) {
        if constexpr (kVec == 4) {
          const float4 x = *reinterpret_cast<const float4*>(src + e);
          v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        } else {
          const float2 x = *reinterpret_cast<const float2*>(src + e);
          v[2 * q] = x.x; v[2 * q + 1] = x.y;
        }
      }
    }
  }

  __device__ __forceinline__ void store(float* ring, int T, int k, int lane) {
    const int row0 = 4 * k + 1;
    if (row0 >= T) return;
    const int lim = ((T - row0) < kChunk ? (T - row0) : kChunk) * STRIDE;
    float* dst = ring + ((4 * k) % kRing) * STRIDE;
#pragma unroll
    for (int q = 0; q < kPer / kVec; ++q) {
      const int e = kVec * (lane + kWave * q);
      if (e < lim) {
        if constexpr (kVec == 4)
          *reinterpret_cast<float4*>(dst + e) = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        else
          *reinterpret_cast<float2*>(dst + e) = make_float2(v[2 * q], v[2 * q + 1]);
      }
    }
  }

  // Pull the cache lines of chunk k into L2 (one dword per 128-byte line).
  __device__ __forceinline__ uint32_t touch(const float* em, int T, int k, int lane) {
    const int row0 = 4 * k + 1;
    const int rows = (T - row0) < kChunk ? (T - row0) : kChunk;
    if (rows > 0 && lane * 32 < rows * STRIDE)
      return __builtin_bit_cast(uint32_t, em[(int64_t)row0 * STRIDE + lane * 32]);
    return 0u;
  }
};

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
template <int M, int STRIDE>
__device__ FwdOut segment_forward(const Inst& in, const int w, const int lane, float* ring,
                                  SegSync* sy, bool labels_bad) {
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
  uint64_t skip[M / 2];   // lane mask per label slot: may enter from two states below
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
    skip[jj] = __builtin_amdgcn_ballot_w64(sk);
  }

  // a3: frame 0.  Only states 0 and 1 start finite.
  float a[M];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int s = sbase + j;
    a[j] = neg_inf();
    if (s == 0) a[j] = em[blank];
    if (s == 1 && S > 1) a[j] = em[in.lab[0]];
  }

  const bool has_next = w + 1 < W, has_prev = w > 0;
  SegSync* me = sy + w;
  SegSync* prev = has_prev ? sy + w - 1 : nullptr;
  SegSync* next = has_next ? sy + w + 1 : nullptr;
  if (has_next) {
    if (lane == kWave - 1) me->bnd[0] = a[M - 1];
    lds_store_rel(&me->prod, 1);
  }

  const int nsteps = T - 1;               // frames 1..T-1
  const int nblk = (int)bp_blocks(T);
  const int NP = bp_planes(M);
  uint32_t* bpw = in.bp + (int64_t)w * nblk * NP * kWave + lane;

  Stager<STRIDE> st;
  uint32_t warm_acc = 0, warm_a = 0, warm_b = 0;
  // Invariant at the switch to chunk k: the stager holds chunk k, warm_a is
  // the touch of chunk k+1 (issued two switches ago, older than the load of
  // chunk k, so already complete) and warm_b the touch of chunk k+2.
  if (nsteps > 0) {
    st.load(em, T, 0, lane);
    warm_b = st.touch(em, T, 2, lane);
  }

  uint32_t mv[M], sk[M / 2];
#pragma unroll
  for (int j = 0; j < M; ++j) mv[j] = 0;
#pragma unroll
  for (int j = 0; j < M / 2; ++j) sk[j] = 0;

  bool alive = true;
  int u = 0;
  for (int b = 0; b < nblk && alive; ++b) {
    const int n = (nsteps - 32 * b) < kBlk ? (nsteps - 32 * b) : kBlk;
    // cross-segment flow control, once per 32-frame block
    if (has_prev) alive &= wait_geq(&prev->prod, 32 * b + n);
    if (has_next && 32 * b + n - kBnd + 1 > 0) alive &= wait_geq(&next->cons, 32 * b + n - kBnd + 1);
    if (!alive) break;

#pragma unroll 1
    for (int g = 0; g < kBlk / kUnroll; ++g) {
#pragma unroll
      for (int i = 0; i < kUnroll; ++i) {
        const int ib = g * kUnroll + i;          // frame index inside the block
        if (ib < n) {
          u = 32 * b + ib;                       // computes frame t = u + 1
          if (i % kChunk == 0) {
            // a2: chunk u/4 is staged in registers; land it, fetch the next
            const int k = u / kChunk;
            st.store(ring, T, k, lane);
            warm_acc ^= warm_a;
            warm_a = warm_b;
            st.load(em, T, k + 1, lane);
            warm_b = st.touch(em, T, k + 3, lane);
          }
          const float* row = ring + (i % kRing) * STRIDE;  // u % 8 == i
          const float eb = row[blank];
          float e[M / 2];
#pragma unroll
          for (int jj = 0; jj < M / 2; ++jj) e[jj] = row[eoff[jj]];
          const float nb_in = has_prev ? prev->bnd[u % kBnd] : neg_inf();
          const float nb = shr1(a[M - 1], nb_in);
          dp_frame<M>(a, mv, sk, skip, nb, eb, e);
          if (has_next && lane == kWave - 1) me->bnd[(u + 1) % kBnd] = a[M - 1];
        }
      }
    }

    // a5: flush this block's backpointer words (frame i of the block at bit 31-i)
    const int sh = kBlk - n;
    uint32_t* dst = bpw + (int64_t)b * NP * kWave;
#pragma unroll
    for (int jj = 0; jj < M / 2; ++jj) {
      dst[(3 * jj) * kWave] = mv[2 * jj] << sh;
      dst[(3 * jj + 1) * kWave] = mv[2 * jj + 1] << sh;
      dst[(3 * jj + 2) * kWave] = sk[jj] << sh;
    }
    if (has_next) lds_store_rel(&me->prod, 32 * b + n + 1);
    if (has_prev) lds_store_rel(&me->cons, 32 * b + n);
  }
  out.ok = alive ? 1 : 0;
  if (warm_acc == 0x7fc00001u && T < 0) in.path[0] = (int)warm_acc;   // keeps the warm-up loads

  // a6: end state, in the segment that holds S-1 and S-2
  if (w == W - 1) {
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
__device__ bool prologue_check(const Inst& in, int w, int lane) {
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
// backpointer block.  Over one block the state drops by at most 62, so the
// block's codes for the 63 states at and below the block's top state sit one
// per lane ("band") and each frame costs three readlanes.  The next block's
// band is fetched before the chase (a 128-state window that covers any exit
// state) and realigned with ds_bpermute once the exit state is known.

struct Band {
  uint32_t mv, sk;
  int lab;
};

__device__ __forceinline__ Band load_band(const Inst& in, int blk, int nblk, int top, int x0, int lane) {
  Band r{0u, 0u, in.blank};
  const int q = top - x0 - lane;
  if (q < 0 || blk < 0) return r;
  const int M = in.M, NP = bp_planes(M);
  const int segsz = kWave * M;
  const int wseg = q / segsz;
  const int rr = q - wseg * segsz;
  const int ln = rr / M;
  const int j = rr - ln * M;
  const uint32_t* base = in.bp + (((int64_t)wseg * nblk + blk) * NP) * kWave + ln;
  if (j % 2 == 0) {
    r.mv = base[(3 * (j / 2)) * kWave];
  } else {
    r.mv = base[(3 * (j / 2) + 1) * kWave];
    r.sk = base[(3 * (j / 2) + 2) * kWave];
    r.lab = in.lab[(q - 1) / 2];
  }
  return r;
}

__device__ __forceinline__ uint32_t bperm(uint32_t v, int src_lane) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane * 4, (int)v);
}

__device__ void fill_outputs(const Inst& in, int lane, int path_val, float score_val) {
  for (int t = lane; t < in.T; t += kWave) {
    in.path[t] = path_val;
    in.scores[t] = score_val;
  }
}

__device__ void backtrack(const Inst& in, const FwdOut& fo, int status_in, int lane) {
  const int T = in.T, RS = in.stride, blank = in.blank;   // RS: emission row stride
  const float* em = in.em;
  int status = status_in;
  float total = fo.total;
  if (status == kOk && !fo.ok) status = kEdevice;
  if (status == kOk && total == neg_inf()) status = kEinfeasible;

  if (status != kOk) {
    const float fillv = (status == kEinfeasible) ? neg_inf() : __builtin_nanf("");
    fill_outputs(in, lane, -1, fillv);
    if (status != kEinfeasible) total = __builtin_nanf("");
  } else {
    const int nblk = (int)bp_blocks(T);
    int s = fo.send;
    Band cur = load_band(in, nblk - 1, nblk, s, 0, lane);
    int pend_lab = 0;
    float pend_sc = 0.f;
    int pend_t0 = -1;
    int pend_n = 0;
    for (int b = nblk - 1; b >= 0; --b) {
      const int n = (T - 1 - 32 * b) < kBlk ? (T - 1 - 32 * b) : kBlk;
      const int top = s;
      Band wa{0u, 0u, blank}, wb{0u, 0u, blank};
      if (b > 0) {
        wa = load_band(in, b - 1, nblk, top, 0, lane);
        wb = load_band(in, b - 1, nblk, top, kWave, lane);
      }
      // chase frames t = 32b+n .. 32b+1 (bit 31-i of the block's words)
      int outlab = blank;
      for (int i = n - 1; i >= 0; --i) {
        const int l = top - s;
        const int lab = __builtin_amdgcn_readlane(cur.lab, l);
        outlab = (lane == i) ? lab : outlab;
        const uint32_t m1 = (uint32_t)__builtin_amdgcn_readlane((int)cur.mv, l);
        const uint32_t m2 = (uint32_t)__builtin_amdgcn_readlane((int)cur.sk, l);
        const int bit = 31 - i;
        const int k = ((m2 >> bit) & 1u) ? 2 : (int)((m1 >> bit) & 1u);
        s -= k;
      }
      // outputs of the previous block (its score gathers have had a block's time)
      if (pend_t0 >= 0 && lane < pend_n) {
        in.path[pend_t0 + lane] = pend_lab;
        in.scores[pend_t0 + lane] = pend_sc;
      }
      pend_t0 = 32 * b + 1;
      pend_n = n;
      pend_lab = outlab;
      pend_sc = lane < n ? em[(int64_t)(pend_t0 + lane) * RS + outlab] : 0.f;
      if (b > 0) {
        const int d = top - s;   // 0..64: exit state = top - d
        const int src = (lane + d) & (kWave - 1);
        const bool hi = lane + d >= kWave;
        const uint32_t amv = bperm(wa.mv, src), bmv = bperm(wb.mv, src);
        const uint32_t ask = bperm(wa.sk, src), bsk = bperm(wb.sk, src);
        const int alab = (int)bperm((uint32_t)wa.lab, src), blab = (int)bperm((uint32_t)wb.lab, src);
        cur.mv = hi ? bmv : amv;
        cur.sk = hi ? bsk : ask;
        cur.lab = hi ? blab : alab;
      }
    }
    if (pend_t0 >= 0 && lane < pend_n) {
      in.path[pend_t0 + lane] = pend_lab;
      in.scores[pend_t0 + lane] = pend_sc;
    }
    // frame 0
    if (lane == 0) {
      const int lab0 = (s % 2 == 0) ? blank : in.lab[(s - 1) / 2];
      in.path[0] = lab0;
      in.scores[0] = em[lab0];
    }
  }
  if (lane == 0) {
    if (in.total) *in.total = total;
    if (in.status) *in.status = status;
  }
}

}  // namespace ctca
