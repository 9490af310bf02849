// Host-side state shared by the library's translation units: contexts,
// batched plans, logging, HIP error mapping and small helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/ctcalign.h"
#include "internal.hpp"
#include "tune.hpp"

namespace ctca {

constexpr int64_t kMaxS = 8 * kWave * 64;      // largest trellis one workgroup holds

inline int log_level() {
  static int lv = [] {
    const char* e = std::getenv("CTCALIGN_LOG");
    return e ? std::atoi(e) : 0;
  }();
  return lv;
}

#define CTCA_LOG(lvl, ...)                       \
  do {                                           \
    if (log_level() >= (lvl)) {                  \
      std::fprintf(stderr, "[ctcalign] " __VA_ARGS__); \
      std::fputc('\n', stderr);                  \
    }                                            \
  } while (0)

inline int map_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return CTCALIGN_OK;
  CTCA_LOG(1, "%s: %s", what, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? CTCALIGN_ENOMEM : CTCALIGN_EDEVICE;
}

#define HIP_TRY(expr)                                 \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return map_hip(_e, #expr);  \
  } while (0)

// Device buffer that only grows.
struct Arena {
  void* ptr = nullptr;
  size_t bytes = 0;
  int reserve(size_t need) {
    if (need <= bytes) return CTCALIGN_OK;
    if (ptr) {
      // launches queued earlier may still use the old buffer
      (void)hipDeviceSynchronize();
      (void)hipFree(ptr);
      ptr = nullptr;
      bytes = 0;
    }
    size_t sz = std::max(need, (size_t)1 << 20);
    if (hipMalloc(&ptr, sz) != hipSuccess) {
      ptr = nullptr;
      return CTCALIGN_ENOMEM;
    }
    bytes = sz;
    return CTCALIGN_OK;
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
};

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline int row_stride_for(int C) { return C <= 32 ? 32 : 256; }

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Host-checkable arguments of one alignment.
inline int validate_one(const float* em, int32_t T, int32_t C, const int32_t* labels, int32_t L,
                        int32_t blank, const void* path, const void* scores) {
  if (!em || !path || !scores) return CTCALIGN_EINVAL;
  if (T < 1 || T > (1 << 30) || C < 1 || C > kMaxC || L < 0) return CTCALIGN_EINVAL;
  if (L > 0 && !labels) return CTCALIGN_EINVAL;
  if (blank < 0 || blank >= C) return CTCALIGN_EINVAL;
  if (2 * (int64_t)L + 1 > kMaxS) return CTCALIGN_EINVAL;
  return CTCALIGN_OK;
}

// The allocation-free entry point's per-device scratch array (noalloc.hip):
// noalloc_setup looks up its address on `device` (which must be current)
// once; noalloc_scratch returns it (nullptr before setup or on failure).
int noalloc_setup(int device);
void* noalloc_scratch(int device);

}  // namespace ctca

struct ctcalign_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  ctca::Arena ws;  // backpointer workspace for single alignments
  ctca::Arena pad; // padded emission copies for single alignments
  // ws and pad are shared by every call that brings no workspace of its own,
  // whatever stream it comes on: each such call waits for the previous one
  // (an event recorded on that call's stream) before it touches them
  hipEvent_t arena_ev = nullptr;
  hipStream_t arena_stream = nullptr;
  bool arena_used = false;
  int32_t* h_status = nullptr;   // pinned
  int32_t* d_status = nullptr;
  float* d_total = nullptr;
  ctca::TuneTable tune;
  ctcalign_plan* cached = nullptr;
  uint64_t cached_key = 0;
};

struct ctcalign_plan {
  ctcalign_ctx* ctx = nullptr;
  int32_t n = 0;
  int npacks = 0;
  int grid = 0;
  ctca::Inst* d_insts = nullptr;
  ctca::Pack* d_packs = nullptr;
  ctca::PadDesc* d_pad = nullptr;
  int npad = 0;
  int64_t pad_max = 0;
  int* d_head = nullptr;
  void* d_bp = nullptr;
  size_t bp_bytes = 0;
  void* d_padbuf = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  int64_t* d_trace = nullptr;          // per pack {start, end, hw id} when tracing
  int nlong = 0;                       // instances too large for packs (k_persistent_long)
  int* d_order = nullptr;              // their indices, longest first
  int* d_head_long = nullptr;
  int ncrit = 0;                       // longest chains (k_persistent_crit, parallel branch)
  int* d_crit = nullptr;
  hipStream_t crit_stream = nullptr;   // capture-time only
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // a replay on one stream waits for the last replay on another one: they
  // share the backpointer workspace and the queue heads
  hipEvent_t run_ev = nullptr;
  hipStream_t run_stream = nullptr;
  bool ran = false;
  std::vector<int> pack_order_inst;    // first instance of each pack (host copy, for traces)
};
