// Single alignment without any device allocation: ctcalign_align_noalloc.
//
// The same computation as ctcalign_align_ex (paper Sec. 4, "CTC-based forced
// alignment"), for callers that cannot call hipMalloc (work recorded under
// HIP graph capture, tight serving loops, harnesses that forbid it).  Its
// backpointer words and, when the rows need re-laying out, the padded
// emission copy live in `scratch`, a fixed array in device global memory of
// kScratchBytes, one copy per device for the life of the process.  Every
// call on a device shares that copy: calls that overlap in time on one
// device (on different streams, or from different threads) race on it, and
// the caller must order them.  Nothing in it has to start at zero: a call
// writes every backpointer word and padded row it later reads.
//
// Host code never passes `scratch` itself (in host code the name is only a
// stand-in for the device symbol): noalloc_setup looks up its device address
// once per device, at context creation with the device current, and the
// kernels get that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.hpp"
#include "kernels.hpp"

using namespace ctca;

namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDev = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDev] = {};

}  // namespace

namespace ctca {

int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDev) return CTCALIGN_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return CTCALIGN_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return map_hip(e, "hipGetSymbolAddress(scratch)");
  if (!p) return CTCALIGN_EDEVICE;
  g_scratch[device] = p;
  return CTCALIGN_OK;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDev) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_scratch[device];
}

}  // namespace ctca

extern "C" {

size_t ctcalign_noalloc_scratch_bytes(void) { return kScratchBytes; }

int ctcalign_align_noalloc(ctcalign_ctx* ctx, const float* emission, int32_t T, int32_t C,
                           const int32_t* labels, int32_t L, int32_t blank, int32_t* out_path,
                           float* out_scores, float* out_total, int32_t* out_status,
                           ctcalign_stream stream) {
  if (!ctx) return CTCALIGN_EINVAL;
  int rc = validate_one(emission, T, C, labels, L, blank, out_path, out_scores);
  if (rc) return rc;
  char* scr = static_cast<char*>(noalloc_scratch(ctx->device));
  if (!scr) return CTCALIGN_EDEVICE;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);

  Inst in{};
  in.T = T;
  in.C = C;
  in.L = L;
  in.blank = blank;
  in.lab = labels;
  in.path = out_path;
  in.scores = out_scores;
  in.total = out_total;
  in.status = out_status;
  in.stride = row_stride_for(C);
  in.prio = 0;
  // one workgroup: the multi-workgroup layout needs its sync region, which
  // lives in memory allocated on first use
  const int S = 2 * L + 1;
  Geo g = ctx->tune.pick_one(S, C);
  if (geometry_is_multi(g.W, g.M)) g = ctx->tune.pick_long(S);
  in.W = g.W;
  in.M = g.M;
  if (!geometry_supported_one_wg(in.W, in.M) || !geo_ok(S, in.W, in.M)) return CTCALIGN_EINVAL;

  const size_t bp_bytes = round_up((size_t)bp_words(T, in.W, in.M) * 4, 256);
  const bool padded = !(C == in.stride && aligned16(emission));
  const size_t pad_bytes = padded ? round_up((size_t)T * in.stride * sizeof(float), 256) : 0;
  if (bp_bytes > kScratchBytes || pad_bytes > kScratchBytes - bp_bytes) {
    CTCA_LOG(1, "align_noalloc: T=%d L=%d C=%d needs %zu bytes of scratch, %zu available", T, L, C,
             bp_bytes + pad_bytes, kScratchBytes);
    return CTCALIGN_ENOMEM;
  }
  in.bp = reinterpret_cast<uint32_t*>(scr);
  if (padded) {
    float* dst = reinterpret_cast<float*>(scr + bp_bytes);
    const PadDesc pd{emission, dst, T, C, in.stride, 0};
    HIP_TRY(launch_pad_one(pd, st));
    in.em = dst;
  } else {
    in.em = emission;
  }
  HIP_TRY(launch_one(in, st));
  return CTCALIGN_OK;
}

}  // extern "C"
