// gfx950 kernels for CTC forced alignment and their host-side launchers.
//
//   k_one<STRIDE>        one instance, W <= 4 waves, M <= 16 states per lane
//   k_one_long<STRIDE>   one instance, W <= 16 waves, 8 <= M <= 32 (long form)
//   k_persistent         batched: each 4-wave workgroup pops work items
//                        ("packs") from a device queue until it is empty
//   k_fill               small fill kernel (queue reset inside graphs)
//
// STRIDE is the LDS row stride of the emission ring: 32 for C <= 32 and 256
// for 32 < C <= 256.
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "kernels.hpp"

namespace ctca {

// Runs segment w of `in` on the calling wave: label check, one workgroup
// barrier, forward pass, then either "done" publication (lower segments) or
// end-state selection and backtrack (the top segment).
template <int M, int STRIDE>
__device__ void run_wave(const Inst& in, int w, int lane, SegSync* sy, float* ring) {
  const bool bad = prologue_check<M>(in, w, lane);
  if (bad && lane == 0) sy[w].bad = 1;
  __syncthreads();
  bool any_bad = false;
  for (int k = 0; k < in.W; ++k) any_bad |= (sy[k].bad != 0);
  const FwdOut fo = segment_forward<M, STRIDE>(in, w, lane, ring, sy, any_bad);
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
    backtrack(in, f2, any_bad ? kEinval : kOk, lane);
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
    run_wave<MM, STRIDE>(in, w, lane, sy, ring); \
    break;

template <int STRIDE>
__global__ void __launch_bounds__(256) k_one(Inst in) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  SegSync* sy = reinterpret_cast<SegSync*>(smem);
  float* ring = reinterpret_cast<float*>(smem + in.W * sizeof(SegSync)) + w * kRing * STRIDE;
  reset_sync(sy + w, lane);
  switch (in.M) {
    CTCA_CASE(2) CTCA_CASE(4) CTCA_CASE(6) CTCA_CASE(8)
    CTCA_CASE(10) CTCA_CASE(12) CTCA_CASE(14) CTCA_CASE(16)
    default: __syncthreads(); break;
  }
}

template <int STRIDE>
__global__ void __launch_bounds__(1024) k_one_long(Inst in) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  SegSync* sy = reinterpret_cast<SegSync*>(smem);
  float* ring = reinterpret_cast<float*>(smem + in.W * sizeof(SegSync)) + w * kRing * STRIDE;
  reset_sync(sy + w, lane);
  switch (in.M) {
    CTCA_CASE(8) CTCA_CASE(12) CTCA_CASE(16) CTCA_CASE(20)
    CTCA_CASE(24) CTCA_CASE(28) CTCA_CASE(30) CTCA_CASE(32)
    default: __syncthreads(); break;
  }
}
#undef CTCA_CASE

template <int STRIDE>
__device__ __forceinline__ void pack_dispatch(const Inst& in, int w, int lane, SegSync* sy, float* ring) {
  switch (in.M) {
    case 2: run_wave<2, STRIDE>(in, w, lane, sy, ring); break;
    case 4: run_wave<4, STRIDE>(in, w, lane, sy, ring); break;
    case 6: run_wave<6, STRIDE>(in, w, lane, sy, ring); break;
    case 8: run_wave<8, STRIDE>(in, w, lane, sy, ring); break;
    case 12: run_wave<12, STRIDE>(in, w, lane, sy, ring); break;
    case 16: run_wave<16, STRIDE>(in, w, lane, sy, ring); break;
    default: __syncthreads(); break;
  }
}

// LDS: [4] SegSync, then 4 rings of kRing*256 floats.
__global__ void __launch_bounds__(256) k_persistent(const Inst* __restrict__ insts,
                                                    const Pack* __restrict__ packs, int npacks,
                                                    int* __restrict__ head) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ int s_item;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  SegSync* sy = reinterpret_cast<SegSync*>(smem);
  float* ring = reinterpret_cast<float*>(smem + kPackWaves * sizeof(SegSync)) + wv * kRing * kMaxC;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(head, 1);
    reset_sync(sy + wv, lane);
    __syncthreads();
    const int item = s_item;
    if (item >= npacks) break;
    const int ii = packs[item].inst[wv];
    if (ii < 0) {
      __syncthreads();   // the barrier the busy waves take inside run_wave
    } else {
      const Inst in = insts[ii];
      const int seg = packs[item].seg[wv];
      const int first = packs[item].first[wv];
      set_prio(in.prio);
      if (in.stride == 32)
        pack_dispatch<32>(in, seg, lane, sy + first, ring);
      else
        pack_dispatch<256>(in, seg, lane, sy + first, ring);
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();     // every wave is done with this pack's LDS
  }
}

// Copies rows of a [T][C] emission into a [T][stride] buffer (zeros in the
// pad columns), so the alignment kernels always see 16-byte aligned rows of
// a compiled stride.  blockIdx.y selects the descriptor.
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

__global__ void k_fill(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---- launchers ---------------------------------------------------------------

size_t lds_bytes_one(int W, int stride) {
  return (size_t)W * sizeof(SegSync) + (size_t)W * kRing * stride * sizeof(float);
}

size_t lds_bytes_persistent() {
  return (size_t)kPackWaves * sizeof(SegSync) + (size_t)kPackWaves * kRing * kMaxC * sizeof(float);
}

static bool m_in(int M, const int* menu, int n) {
  for (int i = 0; i < n; ++i)
    if (menu[i] == M) return true;
  return false;
}

bool geometry_supported_one(int W, int M) {
  static const int small[] = {2, 4, 6, 8, 10, 12, 14, 16};
  static const int large[] = {8, 12, 16, 20, 24, 28, 30, 32};
  if (W >= 1 && W <= 4 && m_in(M, small, 8)) return true;
  if (W >= 1 && W <= 16 && m_in(M, large, 8)) return true;
  return false;
}

bool geometry_supported_pack(int W, int M) {
  static const int menu[] = {2, 4, 6, 8, 12, 16};
  return (W == 1 || W == 2 || W == 4) && m_in(M, menu, 6);
}

static hipError_t set_lds_limit(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_one(const Inst& in, hipStream_t st) {
  const size_t lds = lds_bytes_one(in.W, in.stride);
  static const int small[] = {2, 4, 6, 8, 10, 12, 14, 16};
  const bool use_small = in.W <= 4 && m_in(in.M, small, 8);
  const dim3 block(kWave * in.W);
  hipError_t e;
  if (use_small) {
    if (in.stride == 32) {
      e = set_lds_limit((const void*)k_one<32>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_one<32>, dim3(1), block, lds, st, in);
    } else {
      e = set_lds_limit((const void*)k_one<256>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_one<256>, dim3(1), block, lds, st, in);
    }
  } else {
    if (in.stride == 32) {
      e = set_lds_limit((const void*)k_one_long<32>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_one_long<32>, dim3(1), block, lds, st, in);
    } else {
      e = set_lds_limit((const void*)k_one_long<256>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_one_long<256>, dim3(1), block, lds, st, in);
    }
  }
  return hipGetLastError();
}

hipError_t launch_persistent(const Inst* d_insts, const Pack* d_packs, int npacks, int* d_head,
                             int grid, hipStream_t st) {
  const size_t lds = lds_bytes_persistent();
  hipError_t e = set_lds_limit((const void*)k_persistent, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_persistent, dim3(grid), dim3(kWave * kPackWaves), lds, st, d_insts, d_packs,
                     npacks, d_head);
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

hipError_t launch_fill(int* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

int persistent_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent, kWave * kPackWaves,
                                                   lds_bytes_persistent()) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace ctca
