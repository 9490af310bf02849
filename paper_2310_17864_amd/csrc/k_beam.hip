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
// Layout: one wavefront (a 64-thread workgroup) per utterance, longest
// first, so a frame's steps need no workgroup barrier: lanes exchange values
// by ballot, readlane and wave reductions, and LDS accesses of one wave are
// ordered.  The beam (up to 16 hypotheses) and the frame's row (up to 1024
// classes, 16 per lane) in LDS.  A
// hypothesis's labels live in a tree of nodes in global memory (one node per
// extension, (parent node, label)); prefixes are compared by length and a
// 64-bit hash, confirmed by the node identity or, if the nodes differ, a
// walk up both chains, so equality is exact.
//
// Selection per frame: any B distinct candidates bound the B-th best key
// from below; the bound is the B-th best among the stays and each
// hypothesis's extension by the frame's most probable class.  Only the
// classes whose probability times the beam's largest factor reaches the
// bound are paired with the hypotheses, and only candidates at or above the
// bound enter an LDS list; the top B are ranked by counting (up to 64) or by
// repeated maximum (a longer list); if the list overflows, the top B are
// picked by repeated maximum over all candidates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ctx.hpp"

#pragma clang fp contract(off)

namespace ctca {
namespace {

constexpr int kBT = 64;           // threads per workgroup: one wavefront per utterance
constexpr int kBMaxB = 16;        // beam width limit
constexpr int kBMaxV = 1024;      // class count limit
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

// Wavefront-wide operations (all 64 lanes active).  The reductions are the
// ROCm device library's (DPP within rows, then across them).
extern "C" __device__ __attribute__((const)) float __ockl_wfred_max_f32(float);
extern "C" __device__ __attribute__((const)) unsigned long long __ockl_wfred_max_u64(unsigned long long);
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
// set bits of m below this lane
__device__ __forceinline__ int below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint64_t wave_max(uint64_t v) { return __ockl_wfred_max_u64(v); }
// v of lane q (uniform q), broadcast by two v_readlane
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int q) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, q);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), q);
  return ((uint64_t)hi << 32) | lo;
}

// Global-memory views (plain global loads and stores: their completion is
// not tied to the LDS counter the frame's steps wait on).
typedef __attribute__((address_space(1))) const float gf32_t;
typedef __attribute__((address_space(1))) const uint64_t gcu64_t;   // a node (int2) as one word
typedef __attribute__((address_space(1))) uint64_t gu64_t;
typedef __attribute__((address_space(1))) int32_t gi32_t;
__device__ __forceinline__ int node_parent(uint64_t nd) { return (int)(uint32_t)nd; }
__device__ __forceinline__ int node_label(uint64_t nd) { return (int)(uint32_t)(nd >> 32); }

// Two node chains spell the same labels (exact; the caller has matched the
// lengths and hashes)
__device__ __noinline__ bool same_chain(int a, int b, gcu64_t* nodes) {
  while (a != b) {
    if (a < 0 || b < 0) return false;
    const uint64_t na = nodes[a], nb = nodes[b];
    if (node_label(na) != node_label(nb)) return false;
    a = node_parent(na);
    b = node_parent(nb);
  }
  return true;
}

struct Shared {
  float row[kBMaxV];
  Hyp hyp[kBMaxB];
  int child_of[kBMaxB];                 // beam index of h_j's parent prefix, or -1
  uint32_t merged[kBMaxB][kBMaxV / 32]; // (i, c): h_i + c is a beam hypothesis
  uint64_t list[kBList + 8];            // (+8: zeros read past the count)
  uint64_t bkey[2 * kBMaxB];            // stay keys, then extension keys (0 past n)
  uint64_t win[kBMaxB];
  float spb[kBMaxB], spnb[kBMaxB];      // p_b', p_nb' of the stays
  int16_t vc[kBMaxV];                   // the frame's classes that can reach the bound
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

// Key index of candidate (i, c): i * 1024 + c orders the candidates as
// i * V + c does (c < V <= 1024), without a division to decode it.
__device__ __forceinline__ int cand_idx(int i, int c) { return (i << 10) | c; }

// frames of a 64-frame chunk that blank collapse keeps: not a blank frame
// right after a blank frame (prev: the frame before the chunk was one)
__device__ __forceinline__ uint64_t kept_frames(uint64_t flags, int nt, bool prev) {
  const uint64_t valid = nt >= 64 ? ~0ull : ((1ull << nt) - 1ull);
  return valid & ~(flags & ((flags << 1) | (prev ? 1ull : 0ull)));
}

// KC: class columns per lane (c = lane + 64k, k < KC), KC*64 >= V.
template <int KC>
__global__ void __launch_bounds__(kBT) k_beam(const BeamDesc* __restrict__ descs, int V, int blank,
                                              int B, float thr, int32_t* __restrict__ out_len,
                                              float* __restrict__ out_logp, float* __restrict__ out_scaled,
                                              int32_t* __restrict__ out_exp, int32_t* __restrict__ out_nhyp,
                                              int32_t* __restrict__ out_nkept,
                                              int32_t* __restrict__ out_status) {
  __shared__ Shared sh;
  const int lane = threadIdx.x;
  const BeamDesc d = descs[blockIdx.x];
  gf32_t* const y = (gf32_t*)d.y;
  const int u = d.u;
  const int T = d.T;
  if (lane == 0) {
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
  __syncthreads();
  int n = 1;
  int E = 0;
  int status = 0;
  int kept = 0;            // frames kept by blank collapse (all of them, also after a failure)
  // this lane's classes: their probabilities for the frame being processed,
  // and prefetched for the next kept frame; -1 past the last class
  float yv[KC], pre[KC];
  int pre_t = -1;
  auto load_row = [&](int t, float (&dst)[KC]) {
    int ln = lane;
    asm volatile("" : "+v"(ln));   // recomputed per row: no long-lived lane masks
    const int64_t base = (int64_t)t * V;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int c = ln + k * kBT;
      const float v = y[base + (c < V ? c : V - 1)];
      dst[k] = c < V ? v : -1.0f;
    }
  };
  // blank probability of frame t0 + lane (0 past the end)
  auto blank_p = [&](int t0) -> float {
    return t0 + lane < T ? y[(int64_t)(t0 + lane) * V + blank] : 0.0f;
  };
  uint64_t flags = ballot(blank_p(0) > thr);   // blank frames of the current chunk
  bool prev_blank = false;                      // the frame before the chunk was a blank frame
  for (int t0 = 0; t0 < T; t0 += kBT) {
    const int nt = T - t0 < kBT ? T - t0 : kBT;
    uint64_t keep = kept_frames(flags, nt, prev_blank);
    const bool last_blank = (flags >> (nt - 1)) & 1ull;
    // the next chunk's blank probabilities: loaded now, compared when needed
    const int t1 = t0 + kBT;
    const float nbp = blank_p(t1);
    if (status != 0) {
      kept += __builtin_popcountll(keep);
      keep = 0ull;
    }
    while (keep != 0ull) {
      const int tt = __builtin_ctzll(keep);
      keep &= keep - 1ull;
      const int t = t0 + tt;
      const int ki = kept++;
      if (status != 0) continue;
      // (a) the row (prefetched when this frame was known in time)
      if (pre_t == t) {
#pragma unroll
        for (int k = 0; k < KC; ++k) yv[k] = pre[k];
      } else {
        load_row(t, yv);
      }
      // the next kept frame, in this chunk or the next: start loading its row
      {
        int tn = -1;
        if (keep != 0ull) {
          tn = t0 + __builtin_ctzll(keep);
        } else if (t1 < T) {
          const uint64_t k1 = kept_frames(ballot(nbp > thr), T - t1, last_blank);
          if (k1 != 0ull) tn = t1 + __builtin_ctzll(k1);
        }
        pre_t = tn;
        if (tn >= 0) load_row(tn, pre);
      }
      // the row into LDS (every slot up to 64*KC); in registers the blank
      // then reads -1 like the slots past the last class, and the frame's
      // most probable non-blank class is the smallest of the largest
      int ln = lane;
      asm volatile("" : "+v"(ln));
      float ymax = -1.0f;
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int c = ln + k * kBT;
        sh.row[c] = yv[k];
        yv[k] = c == blank ? -1.0f : yv[k];
        ymax = yv[k] > ymax ? yv[k] : ymax;
      }
      const float rowmax = __ockl_wfred_max_f32(ymax);
      int cs = 0;
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const uint64_t m = ballot(yv[k] == rowmax);
        if (m != 0ull) {
          cs = k * kBT + __builtin_ctzll(m);
          break;
        }
      }
      // (b) for each h_j the first i whose prefix is h_j's without its last
      // label: hashes compared for every i at once, then for the matches
      // the lengths and nodes, and only on a node mismatch the exact walk
      // (same_chain)
      for (int w = lane; w < n * (kBMaxV / 32); w += kBT) sh.merged[w / (kBMaxV / 32)][w % (kBMaxV / 32)] = 0u;
      Hyp hj = sh.hyp[lane < n ? lane : 0];
      int p = -1;
      {
        // every slot's hash read (broadcast), the matches as a bit mask
        // (slots from n on hold stale entries: masked out)
        uint64_t hash_a[kBMaxB];
#pragma unroll
        for (int i = 0; i < kBMaxB; ++i) hash_a[i] = sh.hyp[i].hash;
        uint32_t mm = 0u;
#pragma unroll
        for (int i = kBMaxB - 1; i >= 0; --i) mm = (mm << 1) | (uint32_t)(hj.phash == hash_a[i]);
        mm &= lane < n ? (1u << n) - 1u : 0u;
        while (mm != 0u) {
          const int i = __builtin_ctz(mm);
          mm &= mm - 1u;
          const int len_i = sh.hyp[i].len, node_i = sh.hyp[i].node;
          if (hj.len == len_i + 1 && (hj.pnode == node_i || same_chain(hj.pnode, node_i, (gcu64_t*)d.nodes))) {
            p = i;
            break;
          }
        }
      }
      if (lane < n) sh.child_of[lane] = p;
      __syncthreads();
      // merged extensions: h_p + last_j is h_j
      if (lane < n && p >= 0) atomicOr(&sh.merged[p][hj.last >> 5], 1u << (hj.last & 31));
      __syncthreads();
      // stay keys, and the extension of each hypothesis by the frame's most
      // probable class unless it joins a stay
      // (the stay as cand(j, blank) computes it, from this lane's h_j and
      // parent index; its p_b', p_nb' kept for the next beam)
      uint64_t sk = 0ull, ek = 0ull;
      if (lane < n) {
        const float pb = hj.s * sh.row[blank];
        float pnb = hj.len > 0 ? hj.pnb * sh.row[hj.last] : 0.0f;
        if (p >= 0) {
          const Hyp& q = sh.hyp[p];
          const float x = (hj.last == q.last ? q.pb : q.s) * sh.row[hj.last];
          pnb = pnb + x;
        }
        sh.spb[lane] = pb;
        sh.spnb[lane] = pnb;
        sk = make_key(pb + pnb, cand_idx(lane, blank));
        if (!((sh.merged[lane][cs >> 5] >> (cs & 31)) & 1u))
          ek = make_key(0.0f + (cs == hj.last ? hj.pb : hj.s) * sh.row[cs], cand_idx(lane, cs));
      }
      // (b2) the bound: the B-th largest of those (up to) 2n distinct
      // candidates' keys -- any B distinct candidates bound the B-th best
      // key from below; 1 (every positive candidate) when there are fewer.
      // Lane q holds key q (0 from lane 2n on); every lane ranks its own.
      // Lane q < 32 holds key q (stays, then extensions; 0 past n) and
      // ranks it against the 2n, read from LDS by broadcast.
      uint64_t bound = 1ull;
      {
        if (lane < kBMaxB) {
          sh.bkey[lane] = sk;
          sh.bkey[kBMaxB + lane] = ek;
        }
        __syncthreads();
        const uint64_t key = lane < 2 * kBMaxB ? sh.bkey[lane] : 0ull;
        int rank = 0;
#pragma unroll 4
        for (int q = 0; q < n; ++q) rank += (sh.bkey[q] > key ? 1 : 0) + (sh.bkey[kBMaxB + q] > key ? 1 : 0);
        const int valid = __builtin_popcountll(ballot(key != 0ull));
        if (valid >= B) {
          const uint64_t at = ballot(key != 0ull && rank == B - 1);   // exactly one lane
          if (at != 0ull) bound = lane_u64(key, __builtin_ctzll(at));
        }
      }
      // (c) candidates at or above the bound into the list, appended in lane
      // order by ballot.  A key at or above the bound needs a total at or
      // above the bound's float part.  Float products are monotone, so the
      // largest factor F = max(s_i, p_b_i) over the beam times y[c] bounds
      // every extension by c (exact pruning, no rounding involved): only
      // the classes with F*y[c] at or above it are paired with the beam.
      const float bound_f = __builtin_bit_cast(float, (uint32_t)(bound >> 32));
      int cnt = 0;
      auto append = [&](bool ok, uint64_t key) {
        const uint64_t m = ballot(ok);
        const int slot = cnt + below(m);
        if (ok && slot < kBList) sh.list[slot] = key;
        cnt += __builtin_popcountll(m);
      };
      append(lane < n && sk != 0ull && sk >= bound, sk);
      const float F = __ockl_wfred_max_f32(lane < n ? (hj.s > hj.pb ? hj.s : hj.pb) : 0.0f);
      int nv = 0;
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        const int c = ln + k * kBT;
        // y > 0: a class with y = 0 (or past the end, or the blank) gives
        // no positive total
        const bool ok = yv[k] > 0.0f && yv[k] * F >= bound_f;
        const uint64_t m = ballot(ok);
        if (ok) sh.vc[nv + below(m)] = (int16_t)c;
        nv += __builtin_popcountll(m);
      }
      __syncthreads();
      if (nv > 0) {
        // pairs (i, m): class vc[m] after h_i, m padded to a power of two
        const int lg = nv <= 1 ? 0 : 32 - __builtin_clz((uint32_t)(nv - 1));
        const int pairs = n << lg;
        for (int b0 = 0; b0 < pairs; b0 += kBT) {
          const int q = b0 + lane, i = q >> lg, m = q & ((1 << lg) - 1);
          bool ok = false;
          uint64_t key = 0ull;
          if (i < n && m < nv) {
            const int c = sh.vc[m];
            const Hyp& h = sh.hyp[i];
            // extension (i, c): p_b' = 0, p_nb' = x, total 0 + x
            const float x = (c == h.last ? h.pb : h.s) * sh.row[c];
            if (x >= bound_f && !((sh.merged[i][c >> 5] >> (c & 31)) & 1u)) {
              key = make_key(0.0f + x, cand_idx(i, c));
              ok = key >= bound;
            }
          }
          append(ok, key);
        }
      }
      __syncthreads();
      // (d) the B best keys, in order
      int nsel;
      if (cnt <= kBT) {
        // rank of each listed key among the listed keys (all distinct),
        // read from LDS by broadcast, 8 at a time (zeros past the count)
        if (lane < 8) sh.list[cnt + lane] = 0ull;
        __syncthreads();
        const uint64_t key = lane < cnt ? sh.list[lane] : 0ull;
        int rank = 0;
        for (int q = 0; q < cnt; q += 8) {
#pragma unroll
          for (int r = 0; r < 8; ++r) rank += sh.list[q + r] > key ? 1 : 0;
        }
        if (lane < cnt && rank < B) sh.win[rank] = key;
        nsel = cnt < B ? cnt : B;
      } else if (cnt <= kBList) {
        uint64_t prev = ~0ull;
        nsel = 0;
        for (int r = 0; r < B; ++r) {
          uint64_t best = 0ull;
          for (int q = lane; q < cnt; q += kBT) {
            const uint64_t k = sh.list[q];
            if (k < prev && k > best) best = k;
          }
          best = wave_max(best);
          if (best == 0ull) break;
          if (lane == 0) sh.win[r] = best;
          prev = best;
          nsel = r + 1;
        }
      } else {
        // the list overflowed: repeated maximum over every candidate
        uint64_t prev = ~0ull;
        nsel = 0;
        for (int r = 0; r < B; ++r) {
          uint64_t best = 0ull;
          if (lane < n && sk < prev && sk > best) best = sk;
#pragma unroll
          for (int k = 0; k < KC; ++k) {
            const int c = ln + k * kBT;
            if (yv[k] < 0.0f) continue;   // past the last class, or the blank
            for (int i = 0; i < n; ++i) {
              float pb, pnb;
              if (!cand(sh, i, c, blank, pb, pnb)) continue;
              const uint64_t key = make_key(pb + pnb, cand_idx(i, c));
              if (key < prev && key > best) best = key;
            }
          }
          best = wave_max(best);
          if (best == 0ull) break;
          if (lane == 0) sh.win[r] = best;
          prev = best;
          nsel = r + 1;
        }
      }
      __syncthreads();
      if (nsel == 0) {   // no candidate with a positive total (uniform)
        status = 2;
        continue;
      }
      // (e) the next beam, rescaled by the best total's power of two
      const int e = frexp_exp(__builtin_bit_cast(float, (uint32_t)(sh.win[0] >> 32)));
      E += e;
      Hyp nh;
      if (lane < nsel) {
        // the winner's p_b', p_nb': a stay's as computed above; an
        // extension's p_b' = 0 and p_nb' = its total (0 + x = x)
        const uint64_t wk = sh.win[lane];
        const int idx = key_index(wk);
        const int i = idx >> 10, c = idx & 1023;
        float pb = 0.0f, pnb = __builtin_bit_cast(float, (uint32_t)(wk >> 32));
        if (c == blank) {
          pb = sh.spb[i];
          pnb = sh.spnb[i];
        }
        nh = sh.hyp[i];
        if (c != blank) {
          const int node = ki * B + lane;
          ((gu64_t*)d.nodes)[node] = ((uint64_t)(uint32_t)c << 32) | (uint32_t)nh.node;
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
      if (lane < nsel) sh.hyp[lane] = nh;
      n = nsel;
      __syncthreads();   // the new beam, and its nodes, visible to every lane
    }
    if (t1 < T) flags = ballot(nbp > thr);
    prev_blank = last_blank;
  }
  // outputs: labels by walking each hypothesis's nodes
  const int B0 = u * B;
  if (lane < B) {
    if (status == 0 && lane < n) {
      const Hyp h = sh.hyp[lane];
      int node = h.node;
      for (int k = h.len - 1; k >= 0; --k) {
        const uint64_t nd = ((gcu64_t*)d.nodes)[node];
        ((gi32_t*)d.tok)[(int64_t)lane * T + k] = node_label(nd);
        node = node_parent(nd);
      }
      out_len[B0 + lane] = h.len;
      const float tot = h.pb + h.pnb;
      if (out_scaled) out_scaled[B0 + lane] = tot;
      if (out_logp) out_logp[B0 + lane] = (float)(log((double)tot) + (double)E * 0.69314718055994530942);
    } else {
      out_len[B0 + lane] = 0;
      if (out_scaled) out_scaled[B0 + lane] = 0.0f;
      if (out_logp) out_logp[B0 + lane] = -__builtin_inff();
    }
  }
  if (lane == 0) {
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
  // class columns per lane: the power of two with 64 * KC >= V
  auto kern = V <= 64 ? k_beam<1> : V <= 128 ? k_beam<2> : V <= 256 ? k_beam<4> : V <= 512 ? k_beam<8> : k_beam<16>;
  hipLaunchKernelGGL(kern, dim3(N), dim3(kBT), 0, st, d_desc, V, blank, beam, threshold, out_len, out_logp,
                     out_scaled, out_exp, out_nhyp, out_nkept, out_status);
  HIP_TRY(hipGetLastError());
  if (!workspace) {
    HIP_TRY(hipEventRecord(ctx->arena_ev, st));
    ctx->arena_stream = st;
    ctx->arena_used = true;
  }
  return CTCALIGN_OK;   // a copy from pageable memory has consumed `descs` on return
}

}  // extern "C"
