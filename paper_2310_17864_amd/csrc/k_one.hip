// Single-alignment kernels and their launcher.
//
//   k_one        one alignment, W <= 4 waves, M <= 16 states per lane
//   k_one_long   one alignment, W <= 8 waves, 16 <= M <= 64
#include "kernels_common.hpp"

namespace ctca {

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
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  reset_sync(sy + w, lane);
  switch (in.M) {
    CTCA_CASE(16) CTCA_CASE(24) CTCA_CASE(32) CTCA_CASE(40)
    CTCA_CASE(48) CTCA_CASE(56) CTCA_CASE(60) CTCA_CASE(64)
    default: __syncthreads(); break;
  }
}

bool geometry_supported_one(int W, int M) {
  if (W >= 1 && W <= 4 && m_in(M, kOneMenu, 8)) return true;
  if (geometry_is_multi(W, M) && W <= kXWaves * kXMaxGroups && m_in(M, kMultiMenu, 8)) return true;
  if (W >= 1 && W <= 8 && m_in(M, kLongMenu, 8)) return true;
  return false;
}

bool geometry_supported_one_wg(int W, int M) {
  return (W >= 1 && W <= 4 && m_in(M, kOneMenu, 8)) || (W >= 1 && W <= 8 && m_in(M, kLongMenu, 8));
}

hipError_t launch_one(const Inst& in, hipStream_t st) {
  const dim3 block(kWave * in.W);
  if (in.W <= 4 && m_in(in.M, kOneMenu, 8))
    hipLaunchKernelGGL(k_one, dim3(1), block, 0, st, in);
  else
    hipLaunchKernelGGL(k_one_long, dim3(1), block, 0, st, in);
  return hipGetLastError();
}

}  // namespace ctca
