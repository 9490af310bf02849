// Geometry choice: how many wavefronts (W) and states per lane (M) an
// alignment of S states gets, for a single launch and inside the batched
// persistent kernel.  Defaults come from a cost model; ctcalign_tune
// replaces the per-bucket choices with measured ones.
#pragma once
#include <stdint.h>
#include <stdlib.h>

#include <vector>

#include "internal.hpp"

namespace ctca {

struct Geo {
  int W, M;
};

// M values compiled into each kernel family.
constexpr int kMenuOne[] = {2, 4, 6, 8, 10, 12, 14, 16};          // k_one, W <= 4
constexpr int kMenuLong[] = {16, 24, 32, 40, 48, 56, 60, 64};     // k_one_long, W <= 8
constexpr int kMenuPack[] = {2, 4, 6, 8, 10, 12, 14, 16};         // k_persistent, W in {1,2,4}
constexpr int kMenuMulti[] = {2, 4, 6, 8, 10, 12, 14, 16};
constexpr int kMenuCrit[] = {4, 6, 8, 10, 12};                      // k_persistent_crit, W <= 8                          // k_multi, 4 < W <= 64

// Geometry is usable iff it covers S and the top segment holds S-1 and S-2
// (the end-state choice reads both from one wavefront's registers).
inline bool geo_ok(int S, int W, int M) {
  const int64_t seg = (int64_t)kWave * M;
  return (int64_t)W * seg >= S && ((int64_t)(W - 1) * seg + 2 <= S || W == 1);
}
// Layouts of single-workgroup kernels may also end on a segment that holds
// S-1 alone: the end-state choice then takes a(S-2) from the boundary ring.
inline bool geo_ok_top1(int S, int W, int M) {
  const int64_t seg = (int64_t)kWave * M;
  return (int64_t)W * seg >= S && ((int64_t)(W - 1) * seg + 1 <= S || W == 1);
}

struct TuneTable {
  int num_cu = 256;
  // states-per-lane target for single launches and for packs (cost model:
  // per-frame time of a wave grows ~ 5.5*M + 12 VALU issues)
  int one_target_m = 6;
  int pack_target_m = 12;
  // measured overrides, indexed by S bucket (S / 64) and stride class
  std::vector<Geo> one_override[2], pack_override[2];

  std::vector<Geo>& table(int kind, int C) { return kind == 0 ? one_override[cls(C)] : pack_override[cls(C)]; }

  void set_range(int kind, int s_lo, int s_hi, int C, Geo g) {
    auto& t = table(kind, C);
    const int b1 = s_hi / kWave;
    if ((int)t.size() <= b1) t.resize(b1 + 1, Geo{0, 0});
    for (int b = s_lo / kWave; b <= b1; ++b) t[b] = g;
  }

  // Defaults, then optional overrides from the environment:
  // CTCALIGN_PACK_TARGET_M, CTCALIGN_CRIT_FRAC (0 disables the critical-chain
  // kernel), CTCALIGN_CRIT_PER_CU.
  void load_default(int cus) {
    num_cu = cus > 0 ? cus : 256;
    if (const char* v = std::getenv("CTCALIGN_PACK_TARGET_M")) pack_target_m = std::atoi(v);
    if (const char* v = std::getenv("CTCALIGN_CRIT_FRAC")) crit_frac = std::atof(v);
    if (const char* v = std::getenv("CTCALIGN_CRIT_PER_CU")) crit_per_cu = std::atof(v);
  }

  static int cls(int C) { return C <= 32 ? 0 : 1; }

  static int menu_up(const int* menu, int n, int need) {
    for (int i = 0; i < n; ++i)
      if (menu[i] >= need) return menu[i];
    return -1;
  }

  Geo pick_one(int S, int C) const {
    const int b = S / kWave;
    const auto& ov = one_override[cls(C)];
    if (b < (int)ov.size() && ov[b].W > 0 && geo_ok(S, ov[b].W, ov[b].M)) return ov[b];
    if (S <= 4 * kWave * 16) {
      int W = (S + kWave * one_target_m - 1) / (kWave * one_target_m);
      W = W < 1 ? 1 : (W > 4 ? 4 : W);
      for (; W >= 1; --W)
        for (int M : kMenuOne)
          if (geo_ok(S, W, M)) return Geo{W, M};
    }
    // larger: spread over several workgroups, few states per lane (the
    // per-frame latency grows with M; more workgroups cost only pipeline fill)
    for (int M : kMenuMulti) {
      const int W = (S + kWave * M - 1) / (kWave * M);
      if (W <= kXWaves * kXMaxGroups && geo_ok(S, W, M)) return Geo{W, M};
    }
    return pick_long(S);
  }

  // One workgroup of up to 8 waves (the batched large-trellis kernel).
  Geo pick_long(int S) const {
    for (int M : kMenuLong)
      for (int W = 8; W >= 1; --W)
        if (geo_ok(S, W, M)) return Geo{W, M};
    return Geo{0, 0};
  }

  Geo pick_pack(int S, int C, int T) const {
    (void)T;
    const int b = S / kWave;
    const auto& ov = pack_override[cls(C)];
    if (b < (int)ov.size() && ov[b].W > 0 && geo_ok(S, ov[b].W, ov[b].M)) return ov[b];
    // fewest waves whose states per lane stay within the target, else the
    // feasible layout with the fewest states per lane
    for (int W : {1, 2, 4, 8})
      for (int M : kMenuPack)
        if (W <= kPackWaves && M <= pack_target_m && geo_ok(S, W, M)) return Geo{W, M};
    Geo best{0, 0};
    for (int W : {8, 4, 2, 1})
      for (int M : kMenuPack)
        if (W <= kPackWaves && geo_ok(S, W, M) && (best.W == 0 || M < best.M)) best = Geo{W, M};
    return best;
  }

  // Serving: S up to the pack limit as in the batched kernel; larger ones
  // take one resident 16-wave workgroup, with the fewest states per lane
  // (from 8) that cover S.
  Geo pick_serve(int S, int C, int T) const {
    if (S <= max_pack_states()) return pick_pack(S, C, T);
    for (int M : kMenuPack) {
      if (M < 8) continue;
      const int W = (S + kWave * M - 1) / (kWave * M);
      if (W <= kServeWaves && geo_ok_top1(S, W, M)) return Geo{W, M};
    }
    return Geo{0, 0};
  }
  int64_t max_serve_states() const { return (int64_t)kServeWaves * kWave * 16; }
  // Serving across several resident workgroups (multi-workgroup layout):
  // 4 states per lane where the top segment can hold S-1 and S-2, else 6 or
  // 8; up to kServeMaxParts workgroups running 8 segments each.
  Geo pick_serve_parts(int S) const {
    for (int M : {4, 6, 8}) {
      const int W = (S + kWave * M - 1) / (kWave * M);
      if (W <= kServePartWaves * kServeMaxParts && geo_ok(S, W, M)) return Geo{W, M};
    }
    return Geo{0, 0};
  }

  // Largest trellis for the pack kernel: every S up to 4 * 64 * 16 has a
  // pack layout (W <= 4 covers them all; W = 8 layouts leave gaps above).
  int64_t max_pack_states() const { return 4 * kWave * 16; }

  // Chain latency model (ns per frame of one alignment, measured alone on
  // MI355X: about 190 + 16 M) and the critical-chain selection.
  double chain_ns(const Inst& in) const { return (double)in.T * (190.0 + 16.0 * in.M); }
  double crit_frac = 0.6;
  double crit_per_cu = 1.0;
  int crit_max() const { return crit_frac > 0 ? (int)(crit_per_cu * num_cu) : 0; }
  Geo pick_crit(int S) const {
    for (int M : kMenuCrit)
      for (int W = 1; W <= 8; ++W)
        if (geo_ok(S, W, M)) return Geo{W, M};
    return Geo{0, 0};
  }

  // relative time of one frame on one wave
  double step_cost(Geo g, int stride) const { return 5.5 * g.M + 12.0 + (stride > 32 ? 2.0 : 0.0); }

  // Issue priority.  The queue is sorted longest first, so the first num_cu
  // packs start together, one per CU, and carry the longest chains of the
  // batch: the critical path.  Their waves (one per SIMD) get s_setprio so
  // they run at nearly the speed of a wave alone on its SIMD while the other
  // waves of the CU take the remaining issue slots.  Packs much shorter than
  // the longest one are left at normal priority.
  int prio_packs_per_cu = 1;
  double prio_min_frac = 0.4;
  void assign_priorities(std::vector<Inst>& insts, const std::vector<Pack>& packs,
                         const std::vector<double>& pack_cost) const {
    if (packs.empty()) return;
    const double top = pack_cost[0];
    const size_t n = std::min(packs.size(), (size_t)num_cu * prio_packs_per_cu);
    for (size_t i = 0; i < n; ++i) {
      if (pack_cost[i] < prio_min_frac * top) break;
      for (int k = 0; k < kPackWaves; ++k)
        if (packs[i].inst[k] >= 0) insts[packs[i].inst[k]].prio = 3;
    }
  }
};

}  // namespace ctca
