// The server's resident kernel (k_serve) and its launcher.
#include "kernels_common.hpp"

namespace ctca {

constexpr uint64_t kServeIdle = ~0ull, kServeExit = ~0ull - 1;

// Workgroup b serves the mailbox box[b]: when its sequence number moves past
// the last one finished, the workgroup copies items[b] into LDS, pads the
// emission rows if asked, runs the item's segments (one per wave, the same
// per-wave engine as the batched kernel), and stores the sequence number
// into ack.  Each alignment raises its own completion flag as it finishes.
// Exits when the host sets *stop, or after idle_limit ticks of the 100 MHz
// clock without work.
__global__ void __launch_bounds__(kWave * kServeWaves)
k_serve(const ServeItem* items, ServeBox* box, const int32_t* stop, uint64_t epoch, int64_t idle_limit) {
  __shared__ SegSync sy[kServeWaves + 1];   // + the incoming copy of a multi-workgroup part
  __shared__ __attribute__((aligned(16))) float ring[kServeWaves][kRing * kMaxC];
  __shared__ uint64_t s_item[sizeof(ServeItem) / 8];
  __shared__ uint64_t s_cmd;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  ServeBox* bx = box + blockIdx.x;
  uint64_t done_seq = 0;                // meaningful in thread 0 only
  if (tid == 0) {
    done_seq = host_load(&bx->ack);
    host_store(&bx->live, epoch);
  }
  int64_t idle0 = (int64_t)__builtin_amdgcn_s_memrealtime();
  int idle_polls = 0;
  for (;;) {
    if (tid == 0) {
      uint64_t seq = host_load(&bx->mail) >> 32;
      uint64_t cmd = kServeIdle;
      if (seq != done_seq) {
        cmd = seq;
      } else if (__hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0 ||
                 (int64_t)__builtin_amdgcn_s_memrealtime() - idle0 > idle_limit) {
        // leave: withdraw `live`, then look at the mailbox once more.  The
        // host posts, then reads `live`; with both sides storing before
        // loading, an item posted now is either seen here or the host sees
        // this workgroup gone (and restarts the kernel).
        host_store(&bx->live, 0);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "");
        seq = host_load(&bx->mail) >> 32;
        if (seq != done_seq) {
          host_store(&bx->live, epoch);
          cmd = seq;
        } else {
          cmd = kServeExit;
        }
      }
      s_cmd = cmd;
    }
    __syncthreads();
    const uint64_t cmd = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(s_cmd >> 32)) << 32) |
                         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)s_cmd);
    __syncthreads();                    // every wave has read s_cmd
    if (cmd == kServeExit) break;
    if (cmd == kServeIdle) {
      // back off: ~3.4 us per s_sleep 127 at 2.4 GHz, up to ~55 us per poll
      const int n = 1 + (idle_polls < 120 ? idle_polls / 8 : 15);
      for (int k = 0; k < n; ++k) __builtin_amdgcn_s_sleep(127);
      ++idle_polls;
      continue;
    }
    // the item was written before its mailbox: read it after the mailbox
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    const uint64_t* src = reinterpret_cast<const uint64_t*>(items + blockIdx.x);
    for (int k = tid; k < (int)(sizeof(ServeItem) / 8); k += kWave * kServeWaves) s_item[k] = host_load(src + k);
    reset_sync(sy + w, lane);
    if (w == 0) reset_sync(sy + kServeWaves, lane);
    __syncthreads();
    const ServeItem* it = reinterpret_cast<const ServeItem*>(s_item);
    const int kind = __builtin_amdgcn_readfirstlane(it->kind);
    if (kind == kItemReset) {
      // a tag no alignment uses, in every word of the sync region
      int* p = reinterpret_cast<int*>(it->xs);
      for (int i = tid; i < (int)(sizeof(XSync) / sizeof(int)); i += kWave * kServeWaves) p[i] = -1;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    } else if (kind == kItemPart) {
      // one workgroup of a multi-workgroup alignment: every part checks the
      // whole transcript, so the verdict needs no exchange
      const Inst in = uniform_inst(&it->inst[0]);
      bool bad = false;
      for (int i = tid; i < in.L; i += kWave * kServeWaves) {
        const int v = in.lab[i];
        bad |= (v < 0) | (v >= in.C) | (v == in.blank);
      }
      bad = __syncthreads_or(bad);
      const int part = __builtin_amdgcn_readfirstlane((int)it->part);
      XSync* xs = it->xs;
      const uint32_t tag = (uint32_t)__builtin_amdgcn_readfirstlane((int)it->xtag);
      // 8 segments per workgroup (2 waves per SIMD: the chain's frames stay
      // short); waves 8..15 idle
      const Ring r{ring[w]};
      if (w < kServePartWaves) {
        switch (in.M) {
          case 4: run_multi<4, kServePartWaves>(in, xs, tag, sy, r, part, w, lane, bad); break;
          case 6: run_multi<6, kServePartWaves>(in, xs, tag, sy, r, part, w, lane, bad); break;
          case 8: run_multi<8, kServePartWaves>(in, xs, tag, sy, r, part, w, lane, bad); break;
          default: break;
        }
      }
    } else if (__builtin_amdgcn_readfirstlane(it->npad)) {
      // emission rows into the compiled stride (zeros in the pad columns)
      const PadDesc pd = it->pad;
      const int64_t n = (int64_t)pd.T * pd.stride;
      for (int64_t i = tid; i < n; i += kWave * kServeWaves) {
        const int64_t t = i / pd.stride;
        const int c = (int)(i - t * pd.stride);
        pd.dst[i] = c < pd.C ? pd.src[t * pd.C + c] : 0.f;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (kind == kItemSegments) {
      const int wi = __builtin_amdgcn_readfirstlane((int)it->which[w]);
      if (wi < 0) {
        __syncthreads();   // the barrier the busy waves take inside run_wave
      } else {
        const Inst in = uniform_inst(&it->inst[wi]);
        const int seg = __builtin_amdgcn_readfirstlane((int)it->seg[w]);
        const int first = __builtin_amdgcn_readfirstlane((int)it->first[w]);
        pack_dispatch(in, seg, lane, sy + first, Ring{ring[w]});
      }
    }
    __syncthreads();                    // the item's LDS is free again
    if (tid == 0) {
      done_seq = cmd;
      host_store(&bx->ack, cmd);
    }
    idle0 = (int64_t)__builtin_amdgcn_s_memrealtime();
    idle_polls = 0;
  }
}

hipError_t launch_serve(const ServeItem* d_items, ServeBox* d_box, const int32_t* d_stop,
                        uint64_t epoch, int64_t idle_limit, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_serve, dim3(grid), dim3(kWave * kServeWaves), 0, st, d_items, d_box, d_stop,
                     epoch, idle_limit);
  return hipGetLastError();
}

bool geometry_supported_serve(int W, int M) {
  return W >= 1 && W <= kServeWaves && m_in(M, kPackMenuK, 8);
}

bool geometry_supported_serve_parts(int W, int M) {
  return W > 0 && W <= kServePartWaves * kServeMaxParts && W <= kXWaves * kXMaxGroups &&
         m_in(M, kServePartMenu, 3);
}

}  // namespace ctca
