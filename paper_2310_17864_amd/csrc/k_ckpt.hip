// Checkpointed long form (memory-bounded): the two passes of one long
// alignment in the multi-workgroup layout (CkArgs).
//
//   mode kModeCkFirst  the whole alignment forward, keeping the column of
//                      every K-th frame, no backpointers; end state, total
//                      and status (and on failure the filled outputs)
//   mode kModeCkSeg    one K-frame stretch again from its column, with its
//                      backpointers, backtracked from the state the next
//                      stretch ended on
#include "kernels_common.hpp"

namespace ctca {

__global__ void __launch_bounds__(kWave * kXWaves) k_multi_ck(Inst in, XSync* xs, uint32_t tag, CkArgs ck,
                                                              int mode) {
  __shared__ SegSync sy[kXWaves + 1];   // + the copy of the incoming boundary
  __shared__ __attribute__((aligned(16))) float ring[kXWaves][kRing * kMaxC];
  // a stretch runs only after a first pass (and the later stretches) that
  // succeeded; the flag was written by an earlier launch, so every
  // workgroup reads the same value
  if (mode == kModeCkSeg && __builtin_amdgcn_readfirstlane(ck.state[1]) != 0) return;
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
  const CkArgs c = ck;
#define CTCA_CK_CASE(MM)                                                                     \
  case MM:                                                                                   \
    if (mode == kModeCkFirst)                                                                \
      run_multi<MM, kXWaves, kModeCkFirst>(in, xs, tag, sy, r, g, wl, lane, bad, &c);      \
    else                                                                                     \
      run_multi<MM, kXWaves, kModeCkSeg>(in, xs, tag, sy, r, g, wl, lane, bad, &c);        \
    break;
  switch (in.M) {
    CTCA_CK_CASE(2) CTCA_CK_CASE(4) CTCA_CK_CASE(6) CTCA_CK_CASE(8)
    CTCA_CK_CASE(10) CTCA_CK_CASE(12) CTCA_CK_CASE(14) CTCA_CK_CASE(16)
    default: break;
  }
#undef CTCA_CK_CASE
}

bool geometry_supported_ck(int W, int M) {
  return geometry_is_multi(W, M) && W <= kXWaves * kXMaxGroups && m_in(M, kCkMenu, 8);
}

hipError_t launch_multi_ck(const Inst& in, XSync* xs, uint32_t gen, const CkArgs& ck, int mode,
                           hipStream_t st) {
  if (gen < 1 || gen >= (uint32_t)kXGens || in.T > kXMaxT || !geometry_supported_ck(in.W, in.M) ||
      (mode != kModeCkFirst && mode != kModeCkSeg))
    return hipErrorInvalidValue;
  const int groups = (in.W + kXWaves - 1) / kXWaves;
  Inst in_copy = in;
  XSync* xs_copy = xs;
  uint32_t tag = x_gen_tag(gen);
  CkArgs ck_copy = ck;
  int mode_copy = mode;
  void* args[] = {&in_copy, &xs_copy, &tag, &ck_copy, &mode_copy};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_multi_ck), dim3(groups),
                                    dim3(kWave * kXWaves), args, 0, st);
}

}  // namespace ctca
