// Device building blocks shared by the gfx950 kernel files: the per-wave
// driver of one segment (run_wave, run_multi), wave priority, LDS sync reset,
// dispatch on states per lane, loads and stores of fine-grained host memory,
// and the menus of compiled states-per-lane values.
//
// Emission rows sit in LDS with a stride of 256 floats; in HBM their stride
// is 32 (C <= 32) or 256 (32 < C <= 256), padded by the host when needed.
#pragma once
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

// switch case of a kernel whose LDS holds `ring[w]` per wave
#define CTCA_CASE(MM) \
  case MM:            \
    run_wave<MM>(in, w, lane, sy, Ring{ring[w]}); \
    break;

// One segment of a pack member (batched and serving kernels, M <= 16).
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

// ---- multi layout: one long alignment over several workgroups ---------------

__device__ __forceinline__ bool wait_eq_sys(const int* p, int want) {
  for (int n = 0; n < kXSpinLimit; ++n) {
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == want) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

// First pass of the checkpointed long form, top segment: the outcome (as
// the backtrack would report it; on failure the outputs are filled here and
// no stretch runs) and the end state the last stretch starts from.
__device__ __forceinline__ void ck_first_finish(const Inst& in, const FwdOut& fo, int status_in,
                                                int lane, const CkArgs* ck) {
  int status = status_in;
  float total = fo.total;
  if (status == kOk && !fo.ok) status = kEdevice;
  if (status == kOk && total == neg_inf()) status = kEinfeasible;
  if (status != kOk) {
    fill_outputs(in, lane, -1, status == kEinfeasible ? neg_inf() : __builtin_nanf(""));
    if (status != kEinfeasible) total = __builtin_nanf("");
  }
  if (lane == 0) {
    if (in.total) *in.total = total;
    if (in.status) *in.status = status;
    ck->state[0] = fo.send;
    ck->state[1] = status;
  }
}

// Segment w = g * kWG + wl of a multi-workgroup alignment on wave wl of
// workgroup g (kWG waves per workgroup; sy[kWG] holds the incoming copy).
// kMode / ck: the passes of the checkpointed long form (CkArgs).
template <int M, int kWG, int kMode = kModeFull>
__device__ __forceinline__ void run_multi(const Inst& in, XSync* xs, uint32_t tag, SegSync* sy,
                                          const Ring& ring, int g, int wl, int lane, bool bad,
                                          const CkArgs* ck = nullptr) {
  const int w = g * kWG + wl;
  if (w >= in.W) return;
  XLink xl;
  xl.wl = wl;
  xl.tag = tag;
  xl.in_lds = sy + kWG;
  if (wl == 0 && g > 0) xl.in_ch = &xs->ch[g - 1];
  if (wl == kWG - 1 && w + 1 < in.W) xl.out_ch = &xs->ch[g];
  const FwdOut fo = segment_forward<M, true, kMode>(in, w, lane, ring, sy, bad, xl, ck);
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
    if constexpr (kMode == kModeCkFirst) {
      ck_first_finish(in, f2, bad ? kEinval : kOk, lane, ck);
    } else if constexpr (kMode == kModeCkSeg) {
      // a stretch: the first pass settled the outcome (only an expired wait
      // can still fail it); start where the stretch after this one ended
      f2.total = 0.0f;
      f2.send = __builtin_amdgcn_readfirstlane(ck->state[0]);
      backtrack<M>(in, f2, kOk, lane, ck->state);
      if (!ok && lane == 0) ck->state[1] = kEdevice;
    } else {
      backtrack<M>(in, f2, bad ? kEinval : kOk, lane);
    }
  }
}

// ---- fine-grained host memory ------------------------------------------------

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

// ---- compiled states-per-lane menus ------------------------------------------

inline bool m_in(int M, const int* menu, int n) {
  for (int i = 0; i < n; ++i)
    if (menu[i] == M) return true;
  return false;
}

constexpr int kOneMenu[] = {2, 4, 6, 8, 10, 12, 14, 16};         // k_one, W <= 4
constexpr int kLongMenu[] = {16, 24, 32, 40, 48, 56, 60, 64};    // k_one_long, k_persistent_long
constexpr int kPackMenuK[] = {2, 4, 6, 8, 10, 12, 14, 16};       // k_persistent, k_serve
constexpr int kMultiMenu[] = {2, 4, 6, 8, 10, 12, 14, 16};       // k_multi
constexpr int kCritMenu[] = {4, 6, 8, 10, 12};                   // k_persistent_crit
constexpr int kServePartMenu[] = {4, 6, 8};                      // k_serve, multi-workgroup parts
constexpr int kCkMenu[] = {2, 4, 6, 8, 10, 12, 14, 16};          // k_multi_ck

}  // namespace ctca
