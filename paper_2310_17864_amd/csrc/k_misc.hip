// Small kernels: emission row re-layout (k_pad, k_pad_one), token spans
// (k_spans) and a fill kernel (queue resets inside graphs, sync-region resets).
#include "kernels_common.hpp"

namespace ctca {

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

// Token spans of a frame path: a span starts at a non-blank frame whose
// class differs from the previous frame's; its index is the number of starts
// before it (wave ballot + popcount, then a prefix over the 16 waves in LDS);
// the starting thread walks the span and folds its scores in frame order.
__global__ void __launch_bounds__(1024) k_spans(const int32_t* __restrict__ path,
                                                const float* __restrict__ scores, int T, int blank,
                                                int max_spans, int32_t* __restrict__ tok,
                                                int32_t* __restrict__ start, int32_t* __restrict__ end,
                                                float* __restrict__ score, int32_t* __restrict__ count) {
  __shared__ int wave_tot[16];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  for (int c0 = 0; c0 < T; c0 += 1024) {
    const int t = c0 + tid;
    int cls = -1;
    bool is_start = false;
    if (t < T) {
      cls = path[t];
      is_start = cls >= 0 && cls != blank && (t == 0 || path[t - 1] != cls);
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(is_start);
    const int before = __builtin_popcountll(m & ((lane ? (~0ull >> (64 - lane)) : 0ull)));
    if (lane == 0) wave_tot[wv] = __builtin_popcountll(m);
    __syncthreads();
    int off = base, tot = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      if (k < wv) off += wave_tot[k];
      tot += wave_tot[k];
    }
    if (is_start) {
      const int idx = off + before;
      int e = t;
      float acc = scores[t];
      while (e + 1 < T && path[e + 1] == cls) {
        ++e;
        acc = acc + scores[e];
      }
      if (idx < max_spans) {
        tok[idx] = cls;
        start[idx] = t;
        end[idx] = e + 1;
        score[idx] = acc;
      }
    }
    __syncthreads();
    if (tid == 0) base += tot;
    __syncthreads();
  }
  if (tid == 0) *count = base;
}

__global__ void k_fill(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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

hipError_t launch_spans(const int32_t* path, const float* scores, int T, int blank, int max_spans,
                        int32_t* tok, int32_t* start, int32_t* end, float* score, int32_t* count,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_spans, dim3(1), dim3(1024), 0, st, path, scores, T, blank, max_spans, tok, start,
                     end, score, count);
  return hipGetLastError();
}

hipError_t launch_fill(int* p, int n, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace ctca
