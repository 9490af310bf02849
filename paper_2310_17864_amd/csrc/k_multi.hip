// One long alignment over several workgroups (the multi layout) and its
// launchers.
#include "kernels_common.hpp"

namespace ctca {

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

hipError_t launch_multi_reset(XSync* xs, hipStream_t st) {
  // every slot, count and flag -1: a tag no launch uses
  const int nwords = (int)(sizeof(XSync) / sizeof(int));
  return launch_fill(reinterpret_cast<int*>(xs), nwords, -1, st);
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

}  // namespace ctca
