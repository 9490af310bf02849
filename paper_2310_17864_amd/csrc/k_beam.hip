// CTC prefix beam search with blank collapse on gfx950, and its C-ABI.
//
// The paper's second GPU CTC kernel (Sec. 4, paragraph "CTC decoder": a
// CUDA beam search decoder parallel over batch, hypotheses and vocabulary,
// with the blank-collapse frame skipping of Sec. 5, "CUDA CTC decoder",
// Table 3).  Lexicon-free prefix beam search without a language model over
// per-frame probabilities (float32):
//
//   beam h_0..h_{n-1} in rank order, each a label prefix with p_b, p_nb;
//   per kept frame y:   s = p_b + p_nb
//     stay h_j:         p_b' = s_j * y[blank],  p_nb' = p_nb_j * y[last_j]
//     extend h_i by c:  x = (c == last_i ? p_b_i : s_i) * y[c]
//                       joins h_j's stay (p_nb'_j + x) when h_i + c == h_j,
//                       else a new prefix with p_b' = 0, p_nb' = x
//   the B candidates of largest total p_b' + p_nb' (> 0) form the next beam,
//   ties by key: stay of h_j = j*V + blank, extension (i, c) = i*V + c;
//   every score is then multiplied by 2^-e (best total = f * 2^e, f in
//   [0.5, 1)) and e added to a running exponent E.
//   Blank collapse: a frame whose blank probability exceeds the threshold is
//   dropped when the frame before it is such a frame too.
//
// All float arithmetic is single multiplies and adds, contraction off, so
// every score, every ranking decision and every label equals a plain
// float32 evaluation in the same order bit for bit.
//
// Layout: one 256-thread workgroup per utterance, longest first; the beam (up to 16
// hypotheses) and the frame's row (up to 1024 classes) in LDS.  A
// hypothesis's labels live in a tree of nodes in global memory (one node per
// extension, (parent node, label)); prefixes are compared by length and a
// 64-bit hash, confirmed by the node identity or, if the nodes differ, a
// walk up both chains, so equality is exact.
//
// Selection per frame: any B distinct candidates bound the B-th best key
// from below; the bound is the B-th best among the stays and each
// hypothesis's extension by the frame's most probable class.  Only
// candidates at or above it enter an LDS list; the top B are ranked by
// counting (a short list) or by repeated maximum (a long one); if the list
// overflows, the whole workgroup picks the top B by repeated maximum over
// all candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ctx.hpp"

#pragma clang fp contract(off)

namespace ctca {
namespace {

constexpr int kBT = 256;          // threads per workgroup
constexpr int kBMaxB = 16;        // beam width limit
constexpr int kBMaxV = 1024;      // class count limit
constexpr int kBCols = kBMaxV / kBT;
constexpr int kBList = 1024;      // candidates above the bound kept in LDS

struct BeamDesc {
  const float* y;        // [T][V]
  int32_t* tok;          // B rows of T labels
  int2* nodes;           // T * B nodes: (parent node or -1, label)
  int32_t T;
  int32_t u;             // the utterance's index in the call (its output slots)
};

struct Hyp {
  float pb, pnb, s;
  int32_t last, len, node, pnode;   // pnode: node of the prefix without its last label
  int32_t pad_;
  uint64_t hash, phash;             // of the prefix, and of the prefix without its last label
};

__device__ __forceinline__ uint64_t hash_ext(uint64_t h, int c) {
  return (h ^ (uint64_t)(uint32_t)(c + 1)) * 0x9E3779B97F4A7C15ull;
}

// x * 2^k in steps of at most 2^126 (exact while the result is normal)
__device__ __forceinline__ float scale_pow2(float x, int k) {
  while (k > 126) { x = x * 0x1p126f; k -= 126; }
  while (k < -126) { x = x * 0x1p-126f; k += 126; }
  return x * __builtin_bit_cast(float, (uint32_t)(k + 127) << 23);
}

// e with x = f * 2^e, f in [0.5, 1), for finite x > 0
__device__ __forceinline__ int frexp_exp(float x) {
  const uint32_t b = __builtin_bit_cast(uint32_t, x);
  const int eb = (int)((b >> 23) & 0xffu);
  if (eb > 0) return eb - 126;
  const uint32_t m = b & 0x7fffffu;
  return (31 - __builtin_clz(m)) - 148;
}

__device__ __forceinline__ uint64_t make_key(float tot, int idx) {
  if (!(tot > 0.0f)) return 0ull;
  return ((uint64_t)__builtin_bit_cast(uint32_t, tot) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)idx);
}
__device__ __forceinline__ int key_index(uint64_t k) { return (int)(0xFFFFFFFFu - (uint32_t)k); }

__device__ __forceinline__ uint64_t wave_max(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}

// v of lane q, broadcast (two v_readlane: no LDS round trip)
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int q) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, q);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), q);
  return ((uint64_t)hi << 32) | lo;
}

// h_j's prefix without its last label equals h_i's prefix (exact)
__device__ bool parent_is(const Hyp& j, const Hyp& i, const int2* nodes) {
  if (j.len != i.len + 1 || j.phash != i.hash) return false;
  int a = j.pnode, b = i.node;
  while (a != b) {
    if (a < 0 || b < 0) return false;
    const int2 na = nodes[a], nb = nodes[b];
    if (na.y != nb.y) return false;
    a = na.x;
    b = nb.x;
  }
  return true;
}

struct Shared {
  float row[kBMaxV];
  Hyp hyp[kBMaxB];
  int child_of[kBMaxB];                 // beam index of h_j's parent prefix, or -1
  uint32_t merged[kBMaxB][kBMaxV / 32]; // (i, c): h_i + c is a beam hypothesis
  uint64_t stay_key[kBMaxB];
  uint64_t ext_key[kBMaxB];             // extension of h_j by the frame's top class
  uint64_t rowmax[kBT / 64];
  uint64_t bound;
  uint64_t list[kBList];
  uint64_t win[kBMaxB];
  uint64_t wmax[2][kBT / 64];
  int cnt, nsel;
  uint8_t flag[kBT];                    // blank-frame flags of the current 256-frame chunk
};

// Candidate (i, c) of the current frame: p_b', p_nb' (stays include the
// extension that joins them).  Returns false for an extension that joins a
// stay (it is part of that stay) -- never for c == blank.
__device__ __forceinline__ bool cand(const Shared& sh, int i, int c, int blank, float& pb, float& pnb) {
  const Hyp& h = sh.hyp[i];
  if (c == blank) {
    pb = h.s * sh.row[blank];
    pnb = h.len > 0 ? h.pnb * sh.row[h.last] : 0.0f;
    const int p = sh.child_of[i];
    if (p >= 0) {
      const Hyp& q = sh.hyp[p];
      const float x = (h.last == q.last ? q.pb : q.s) * sh.row[h.last];
      pnb = pnb + x;
    }
    return true;
  }
  if ((sh.merged[i][c >> 5] >> (c & 31)) & 1u) return false;
  pb = 0.0f;
  pnb = (c == h.last ? h.pb : h.s) * sh.row[c];
  return true;
}

__global__ void __launch_bounds__(kBT) k_beam(const BeamDesc* __restrict__ descs, int V, int blank,
                                              int B, float thr, int32_t* __restrict__ out_len,
                                              float* __restrict__ out_logp, float* __restrict__ out_scaled,
                                              int32_t* __restrict__ out_exp, int32_t* __restrict__ out_nhyp,
                                              int32_t* __restrict__ out_nkept,
                                              int32_t* __restrict__ out_status) {
  __shared__ Shared sh;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const BeamDesc d = descs[blockIdx.x];
  const int u = d.u;
  const int T = d.T;
  if (tid == 0) {
    Hyp h{};
    h.pb = 1.0f;
    h.pnb = 0.0f;
    h.s = 1.0f;
    h.last = -1;
    h.len = 0;
    h.node = -1;
    h.pnode = -1;
    h.hash = 0;
    h.phash = 0;
    sh.hyp[0] = h;
  }
  int n = 1;
  int E = 0;
  int status = 0;
  int kept = 0;            // frames kept by blank collapse (all of them, also after a failure)
  bool prev_blank = false;
  const int words = (V + 31) >> 5;
  // this thread's classes: c = tid + k*256; their probabilities for the
  // frame being processed, and prefetched for the next kept frame
  float yv[kBCols], pre[kBCols];
  int pre_t = -1;
  for (int t0 = 0; t0 < T; t0 += kBT) {
    // blank-frame flags of the next 256 frames, read at once
    const int nt = T - t0 < kBT ? T - t0 : kBT;
    __syncthreads();   // the previous chunk's flags are no longer read
    if (tid < nt) sh.flag[tid] = d.y[(int64_t)(t0 + tid) * V + blank] > thr ? 1 : 0;
    __syncthreads();
    for (int tt = 0; tt < nt; ++tt) {
      const int t = t0 + tt;
      const bool is_blank = sh.flag[tt] != 0;
      const bool keep = !(is_blank && prev_blank);
      prev_blank = is_blank;
      if (!keep) continue;
      const int ki = kept++;
      if (status != 0) continue;
      // (a) the row (prefetched when this frame was known in time)
      if (pre_t == t) {
#pragma unroll
        for (int k = 0; k < kBCols; ++k) yv[k] = pre[k];
      } else {
        const float* yt = d.y + (int64_t)t * V;
#pragma unroll
        for (int k = 0; k < kBCols; ++k) yv[k] = tid + k * kBT < V ? yt[tid + k * kBT] : 0.0f;
      }
      // the next kept frame of this chunk, if any: start loading its row
      {
        int tn = -1;
        bool pb_ = is_blank;
        for (int q = tt + 1; q < nt; ++q) {
          const bool ib = sh.flag[q] != 0;
          if (!(ib && pb_)) { tn = t0 + q; break; }
          pb_ = ib;
        }
        pre_t = tn;
        if (tn >= 0) {
          const float* yn = d.y + (int64_t)tn * V;
#pragma unroll
          for (int k = 0; k < kBCols; ++k) pre[k] = tid + k * kBT < V ? yn[tid + k * kBT] : 0.0f;
        }
      }
#pragma unroll
      for (int k = 0; k < kBCols; ++k)
        if (tid + k * kBT < V) sh.row[tid + k * kBT] = yv[k];
      // the frame's most probable non-blank class (ties: the smaller class)
      {
        uint64_t best = 0ull;
#pragma unroll
        for (int k = 0; k < kBCols; ++k) {
          const int c = tid + k * kBT;
          if (c < V && c != blank) {
            const uint64_t key = ((uint64_t)__builtin_bit_cast(uint32_t, yv[k]) << 32) |
                                 (uint64_t)(0xFFFFFFFFu - (uint32_t)c);
            best = key > best ? key : best;
          }
        }
        best = wave_max(best);
        if (lane == 0) sh.rowmax[wv] = best;
      }
      for (int w = tid; w < n * words; w += kBT) sh.merged[w / words][w % words] = 0u;
      if (tid < n) {
        // the first i whose prefix is h_j's without its last label: length
        // and hash read for every i at once, nodes compared, and only on a
        // node mismatch the exact walk (parent_is)
        const Hyp hj = sh.hyp[tid];
        int p = -1;
#pragma unroll
        for (int i = 0; i < kBMaxB; ++i) {
          const int len_i = sh.hyp[i].len, node_i = sh.hyp[i].node;
          const uint64_t hash_i = sh.hyp[i].hash;
          if (p < 0 && i < n && hj.len == len_i + 1 && hj.phash == hash_i &&
              (hj.pnode == node_i || parent_is(hj, sh.hyp[i], d.nodes)))
            p = i;
        }
        sh.child_of[tid] = p;
      }
      if (tid == 0) sh.cnt = 0;
      __syncthreads();
      // (b) merged extensions; stay keys; the extension of each hypothesis by
      // the frame's most probable class (unless it joins a stay)
      if (tid < n) {
        const int p = sh.child_of[tid];
        if (p >= 0) {
          const int c = sh.hyp[tid].last;
          atomicOr(&sh.merged[p][c >> 5], 1u << (c & 31));
        }
        float pb, pnb;
        cand(sh, tid, blank, blank, pb, pnb);
        sh.stay_key[tid] = make_key(pb + pnb, tid * V + blank);
        uint64_t rm = 0ull;
        for (int w = 0; w < kBT / 64; ++w) rm = sh.rowmax[w] > rm ? sh.rowmax[w] : rm;
        uint64_t ek = 0ull;
        if (rm != 0ull) {
          const int cs = (int)(0xFFFFFFFFu - (uint32_t)rm);
          bool joins = false;
#pragma unroll
          for (int k = 0; k < kBMaxB; ++k) {
            const int ck = sh.child_of[k], lk = sh.hyp[k].last;
            joins |= k < n && ck == tid && lk == cs;
          }
          if (!joins) {
            const Hyp& h = sh.hyp[tid];
            ek = make_key(0.0f + (cs == h.last ? h.pb : h.s) * sh.row[cs], tid * V + cs);
          }
        }
        sh.ext_key[tid] = ek;
      }
      __syncthreads();
      // (b2) the bound: the B-th largest of those (up to) 2n distinct
      // candidates' keys -- any B distinct candidates bound the B-th best
      // key from below; 1 (every positive candidate) when there are fewer
      if (wv == 0) {
        uint64_t key = 0ull;
        if (lane < n) key = sh.stay_key[lane];
        else if (lane < 2 * n) key = sh.ext_key[lane - n];
        // the keys are read once (lane q holds key q) and broadcast by
        // readlane; every lane ranks its own
        int rank = 0;
#pragma unroll
        for (int q = 0; q < 2 * kBMaxB; ++q) rank += (q < 2 * n && lane_u64(key, q) > key) ? 1 : 0;
        const int valid = __builtin_popcountll(__builtin_amdgcn_ballot_w64(key != 0ull));
        if (lane == 0 && valid < B) sh.bound = 1ull;
        if (lane < 2 * n && key != 0ull && rank == B - 1 && valid >= B) sh.bound = key;
      }
      __syncthreads();
      // (c) candidates at or above the bound into the list
      const uint64_t bound = sh.bound;
      if (tid < n && sh.stay_key[tid] != 0ull && sh.stay_key[tid] >= bound) {
        const int slot = atomicAdd(&sh.cnt, 1);
        if (slot < kBList) sh.list[slot] = sh.stay_key[tid];
      }
      // A key at or above the bound needs a total at or above the bound's
      // float part; float products are monotone, so max(s, p_b) times this
      // thread's largest probability bounds every extension of a hypothesis
      // here (exact pruning, no rounding involved).
      const float bound_f = __builtin_bit_cast(float, (uint32_t)(bound >> 32));
      float ymax = 0.0f;
#pragma unroll
      for (int k = 0; k < kBCols; ++k) {
        const int c = tid + k * kBT;
        if (c < V && c != blank) ymax = yv[k] > ymax ? yv[k] : ymax;
      }
      for (int i = 0; i < n; ++i) {
        const Hyp& h = sh.hyp[i];
        const float hs = h.s, hpb = h.pb;
        if ((hs > hpb ? hs : hpb) * ymax < bound_f) continue;
        const int hl = h.last;
#pragma unroll
        for (int k = 0; k < kBCols; ++k) {
          const int c = tid + k * kBT;
          // extension (i, c): p_b' = 0, p_nb' = x, total 0 + x
          const float x = (c == hl ? hpb : hs) * yv[k];
          if (!(x >= bound_f) || c >= V || c == blank) continue;
          if ((sh.merged[i][c >> 5] >> (c & 31)) & 1u) continue;
          const uint64_t key = make_key(0.0f + x, i * V + c);
          if (key >= bound) {
            const int slot = atomicAdd(&sh.cnt, 1);
            if (slot < kBList) sh.list[slot] = key;
          }
        }
      }
      __syncthreads();
      // (d) the B best keys, in order
      const int cnt = sh.cnt;
      if (cnt <= kBT) {
        // rank of each listed key among the listed keys (all distinct)
        if (tid < cnt) {
          const uint64_t key = sh.list[tid];
          int rank = 0;
          for (int j = 0; j < cnt; ++j) rank += sh.list[j] > key ? 1 : 0;
          if (rank < B) sh.win[rank] = key;
        }
        if (tid == 0) sh.nsel = cnt < B ? cnt : B;
      } else if (cnt <= kBList) {
        if (wv == 0) {
          uint64_t prev = ~0ull;
          int m = 0;
          for (int r = 0; r < B; ++r) {
            uint64_t best = 0ull;
            for (int q = lane; q < cnt; q += 64) {
              const uint64_t k = sh.list[q];
              if (k < prev && k > best) best = k;
            }
            best = wave_max(best);
            if (best == 0ull) break;
            if (lane == 0) sh.win[r] = best;
            prev = best;
            m = r + 1;
          }
          if (lane == 0) sh.nsel = m;
        }
      } else {
        // the list overflowed: repeated maximum over every candidate
        uint64_t prev = ~0ull;
        int m = 0;
        for (int r = 0; r < B; ++r) {
          uint64_t best = 0ull;
          if (tid < n && sh.stay_key[tid] < prev && sh.stay_key[tid] > best) best = sh.stay_key[tid];
          for (int k = 0; k < kBCols; ++k) {
            const int c = tid + k * kBT;
            if (c >= V || c == blank) continue;
            for (int i = 0; i < n; ++i) {
              float pb, pnb;
              if (!cand(sh, i, c, blank, pb, pnb)) continue;
              const uint64_t key = make_key(pb + pnb, i * V + c);
              if (key < prev && key > best) best = key;
            }
          }
          best = wave_max(best);
          if (lane == 0) sh.wmax[r & 1][wv] = best;
          __syncthreads();
          best = 0ull;
          for (int w = 0; w < kBT / 64; ++w) best = sh.wmax[r & 1][w] > best ? sh.wmax[r & 1][w] : best;
          if (best == 0ull) break;
          if (tid == 0) sh.win[r] = best;
          prev = best;
          m = r + 1;
        }
        if (tid == 0) sh.nsel = m;
      }
      __syncthreads();
      const int nsel = sh.nsel;
      if (nsel == 0) {   // no candidate with a positive total (uniform)
        status = 2;
        continue;
      }
      // (e) the next beam, rescaled by the best total's power of two
      const int e = frexp_exp(__builtin_bit_cast(float, (uint32_t)(sh.win[0] >> 32)));
      E += e;
      Hyp nh;
      if (tid < nsel) {
        const int idx = key_index(sh.win[tid]);
        const int i = idx / V, c = idx - i * V;
        float pb, pnb;
        cand(sh, i, c, blank, pb, pnb);
        nh = sh.hyp[i];
        if (c != blank) {
          const int node = ki * B + tid;
          d.nodes[node] = make_int2(nh.node, c);
          nh.phash = nh.hash;
          nh.hash = hash_ext(nh.hash, c);
          nh.pnode = nh.node;
          nh.node = node;
          nh.len += 1;
          nh.last = c;
        }
        nh.pb = scale_pow2(pb, -e);
        nh.pnb = scale_pow2(pnb, -e);
        nh.s = nh.pb + nh.pnb;
      }
      __syncthreads();
      if (tid < nsel) sh.hyp[tid] = nh;
      n = nsel;
      __syncthreads();   // new beam and its nodes visible to the whole workgroup
    }
  }
  // outputs: labels by walking each hypothesis's nodes
  const int B0 = u * B;
  if (tid < B) {
    if (status == 0 && tid < n) {
      const Hyp h = sh.hyp[tid];
      int node = h.node;
      for (int k = h.len - 1; k >= 0; --k) {
        const int2 nd = d.nodes[node];
        d.tok[(int64_t)tid * T + k] = nd.y;
        node = nd.x;
      }
      out_len[B0 + tid] = h.len;
      const float tot = h.pb + h.pnb;
      if (out_scaled) out_scaled[B0 + tid] = tot;
      if (out_logp) out_logp[B0 + tid] = (float)(log((double)tot) + (double)E * 0.69314718055994530942);
    } else {
      out_len[B0 + tid] = 0;
      if (out_scaled) out_scaled[B0 + tid] = 0.0f;
      if (out_logp) out_logp[B0 + tid] = -__builtin_inff();
    }
  }
  if (tid == 0) {
    if (out_exp) out_exp[u] = E;
    out_nhyp[u] = status == 0 ? n : 0;
    if (out_nkept) out_nkept[u] = kept;
    out_status[u] = status;
  }
}

// Workspace: [descriptors | nodes]
struct BeamPlan {
  size_t desc_bytes = 0, node_off = 0, bytes = 0;
  std::vector<int64_t> node_of;   // node array offset (int2 elements) per utterance
};

BeamPlan beam_plan(int32_t N, const int32_t* T, int32_t B) {
  BeamPlan p;
  p.desc_bytes = round_up(sizeof(BeamDesc) * (size_t)std::max(N, 1), 256);
  p.node_off = p.desc_bytes;
  p.node_of.resize((size_t)std::max(N, 0));
  int64_t nodes = 0;
  for (int i = 0; i < N; ++i) {
    p.node_of[i] = nodes;
    nodes += (int64_t)T[i] * B;
  }
  p.bytes = p.node_off + round_up(sizeof(int2) * (size_t)std::max<int64_t>(nodes, 1), 256);
  return p;
}

}  // namespace
}  // namespace ctca

using namespace ctca;

extern "C" {

size_t ctcalign_beam_workspace_bytes(int32_t N, const int32_t* T, int32_t beam) {
  if (N < 0 || (N > 0 && !T) || beam < 1 || beam > kBMaxB) return 0;
  for (int i = 0; i < N; ++i)
    if (T[i] < 1) return 0;
  return beam_plan(N, T, beam).bytes;
}

int ctcalign_beam_decode(ctcalign_ctx* ctx, int32_t N, const float* probs, const int64_t* prob_off,
                         const int32_t* T, int32_t V, int32_t blank, int32_t beam, float threshold,
                         int32_t* out_tokens, const int64_t* tok_off, int32_t* out_len,
                         float* out_logp, float* out_scaled, int32_t* out_exp, int32_t* out_nhyp,
                         int32_t* out_nkept, int32_t* out_status, void* workspace, size_t ws_bytes,
                         ctcalign_stream stream) {
  if (!ctx || N < 0 || V < 2 || V > kBMaxV || blank < 0 || blank >= V || beam < 1 ||
      beam > kBMaxB || !(threshold == threshold))
    return CTCALIGN_EINVAL;
  if (N == 0) return CTCALIGN_OK;
  if (!probs || !prob_off || !T || !out_tokens || !tok_off || !out_len || !out_nhyp || !out_status)
    return CTCALIGN_EINVAL;
  for (int i = 0; i < N; ++i)
    if (T[i] < 1 || prob_off[i] < 0 || tok_off[i] < 0) return CTCALIGN_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const BeamPlan p = beam_plan(N, T, beam);
  if (workspace && (ws_bytes < p.bytes || (reinterpret_cast<uintptr_t>(workspace) & 255u)))
    return CTCALIGN_EINVAL;
  char* ws;
  if (workspace) {
    ws = static_cast<char*>(workspace);
  } else {
    // the context's arena, ordered across streams like every call that uses it
    if (!ctx->arena_ev) HIP_TRY(hipEventCreateWithFlags(&ctx->arena_ev, hipEventDisableTiming));
    if (ctx->arena_used && ctx->arena_stream != st) HIP_TRY(hipStreamWaitEvent(st, ctx->arena_ev, 0));
    const int rc = ctx->ws.reserve(p.bytes);
    if (rc) return rc;
    ws = static_cast<char*>(ctx->ws.ptr);
  }
  // workgroups in order of decreasing frame count: the longest serial
  // chains start first and the short ones fill in beside them
  std::vector<int> order(N);
  for (int i = 0; i < N; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return T[a] > T[b]; });
  std::vector<BeamDesc> descs(N);
  int2* nodes = reinterpret_cast<int2*>(ws + p.node_off);
  for (int k = 0; k < N; ++k) {
    const int i = order[k];
    descs[k].y = probs + prob_off[i];
    descs[k].tok = out_tokens + tok_off[i];
    descs[k].nodes = nodes + p.node_of[i];
    descs[k].T = T[i];
    descs[k].u = i;
  }
  BeamDesc* d_desc = reinterpret_cast<BeamDesc*>(ws);
  HIP_TRY(hipMemcpyAsync(d_desc, descs.data(), sizeof(BeamDesc) * N, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_beam, dim3(N), dim3(kBT), 0, st, d_desc, V, blank, beam, threshold, out_len,
                     out_logp, out_scaled, out_exp, out_nhyp, out_nkept, out_status);
  HIP_TRY(hipGetLastError());
  if (!workspace) {
    HIP_TRY(hipEventRecord(ctx->arena_ev, st));
    ctx->arena_stream = st;
    ctx->arena_used = true;
  }
  return CTCALIGN_OK;   // a copy from pageable memory has consumed `descs` on return
}

}  // extern "C"
