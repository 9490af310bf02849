// Batched persistent kernels and their launchers.
//
//   k_persistent        4-wave workgroups pop work items ("packs": one W=4
//                       alignment, two W=2 or four W=1) from a device queue
//                       sorted longest first until it is empty
//   k_persistent_crit   the batch's longest chains, one alignment per 8-wave
//                       workgroup with few states per lane
//   k_persistent_long   trellises above 4096 states, one per 8-wave workgroup
#include "kernels_common.hpp"

namespace ctca {

// LDS: 4 SegSync and, per wave, an 8-row emission ring of the widest stride.
// trace (optional, may be null): per pack {start, end} of the 100 MHz
// wall clock and the hardware id of the CU that ran it.
__global__ void __launch_bounds__(kWave * kPackWaves) __attribute__((amdgpu_waves_per_eu(4)))
k_persistent(const Inst* __restrict__ insts, const Pack* __restrict__ packs, int npacks,
             int* __restrict__ head, int64_t* __restrict__ trace) {
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

bool geometry_supported_pack(int W, int M) {
  return (W == 1 || W == 2 || W == 4 || W == 8) && W <= kPackWaves && m_in(M, kPackMenuK, 8);
}

bool geometry_supported_crit(int W, int M) { return W >= 1 && W <= 8 && m_in(M, kCritMenu, 5); }

bool geometry_supported_long_batch(int W, int M) { return W >= 1 && W <= 8 && m_in(M, kLongMenu, 8); }

hipError_t launch_persistent(const Inst* d_insts, const Pack* d_packs, int npacks, int* d_head,
                             int grid, hipStream_t st, int64_t* d_trace) {
  hipLaunchKernelGGL(k_persistent, dim3(grid), dim3(kWave * kPackWaves), 0, st, d_insts, d_packs,
                     npacks, d_head, d_trace);
  return hipGetLastError();
}

hipError_t launch_persistent_long(const Inst* d_insts, const int* d_order, int n, int* d_head,
                                  int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_persistent_long, dim3(grid), dim3(kWave * 8), 0, st, d_insts, d_order, n,
                     d_head);
  return hipGetLastError();
}

hipError_t launch_persistent_crit(const Inst* d_insts, const int* d_order, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_persistent_crit, dim3(n), dim3(512), 0, st, d_insts, d_order, n);
  return hipGetLastError();
}

int persistent_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent, kWave * kPackWaves, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace ctca
