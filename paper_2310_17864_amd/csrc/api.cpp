// Host side of libctcalign: argument checks, contexts, geometry choice,
// workspace arenas, launches and the batched plan (sorted work queue +
// captured HIP graph).  Every computation runs in the gfx950 kernels; this
// file only prepares descriptors and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ctx.hpp"
#include "kernels.hpp"

using namespace ctca;

namespace {
constexpr int kMaxDevices = 64;
}  // namespace

namespace {

std::mutex g_default_mu;
ctcalign_ctx* g_default[kMaxDevices] = {};

// Sync region of multi-workgroup alignments, one per device, in uncached
// device memory: workgroups on different XCDs poll it, and a cached copy of a
// line in one XCD's L2 would hide the other XCDs' writes.  Kept for the life
// of the process (uncached memory is never freed once a kernel has read it).
// Launches that use it are serialised with an event, whatever stream they
// come on.  Each launch tags what it writes with its own generation, so the
// region is reset only when the generations run out, and then synchronously:
// no launch ever depends on a reset kernel queued just before it.
struct MultiSync {
  std::mutex mu;
  XSync* region = nullptr;
  hipEvent_t last = nullptr;
  bool used = false;
  uint32_t gen = 0;   // generation of the last launch since the last reset
};
MultiSync g_msync[kMaxDevices];

// ck / mode: a pass of the checkpointed long form (launch_multi_ck) instead
// of a whole alignment.
int launch_multi_serial(int device, const Inst& in, hipStream_t st, const CkArgs* ck = nullptr,
                        int mode = kModeFull) {
  if (device < 0 || device >= kMaxDevices) return CTCALIGN_EDEVICE;
  MultiSync& m = g_msync[device];
  std::lock_guard<std::mutex> lk(m.mu);
  if (!m.region) {
    void* p = nullptr;
    HIP_TRY(hipExtMallocWithFlags(&p, sizeof(XSync), hipDeviceMallocUncached));
    m.region = static_cast<XSync*>(p);
    HIP_TRY(hipEventCreateWithFlags(&m.last, hipEventDisableTiming));
    m.gen = kXGens - 1;   // forces the first reset
  }
  if (m.used) HIP_TRY(hipStreamWaitEvent(st, m.last, 0));
  if (m.gen + 1 >= (uint32_t)kXGens) {
    // every earlier launch and the reset itself complete before the next one
    HIP_TRY(launch_multi_reset(m.region, st));
    HIP_TRY(hipStreamSynchronize(st));
    m.gen = 0;
  }
  ++m.gen;
  if (ck)
    HIP_TRY(launch_multi_ck(in, m.region, m.gen, *ck, mode, st));
  else
    HIP_TRY(launch_multi(in, m.region, m.gen, st));
  HIP_TRY(hipEventRecord(m.last, st));
  m.used = true;
  return CTCALIGN_OK;
}

// Fills geometry and LDS stride fields of an Inst for a single launch.
void geometry_one(const ctcalign_ctx* ctx, Inst& in) {
  const int S = 2 * in.L + 1;
  Geo g = ctx->tune.pick_one(S, in.C);
  // the multi-workgroup layout tags frame indices in 21 bits
  if (geometry_is_multi(g.W, g.M) && in.T > kXMaxT) g = ctx->tune.pick_long(S);
  in.W = g.W;
  in.M = g.M;
}

int launch_single(ctcalign_ctx* ctx, const float* emission, int32_t T, int32_t C,
                  const int32_t* labels, int32_t L, int32_t blank, int32_t* out_path,
                  float* out_scores, float* out_total, int32_t* out_status, void* workspace,
                  size_t ws_bytes, hipStream_t st) {
  int rc = validate_one(emission, T, C, labels, L, blank, out_path, out_scores);
  if (rc) return rc;
  Inst in{};
  in.T = T;
  in.C = C;
  in.L = L;
  in.blank = blank;
  in.lab = labels;
  in.path = out_path;
  in.scores = out_scores;
  in.total = out_total;
  in.status = out_status;
  in.stride = row_stride_for(C);
  in.prio = 0;
  geometry_one(ctx, in);
  if (!geometry_supported_one(in.W, in.M) || !geo_ok(2 * L + 1, in.W, in.M)) return CTCALIGN_EINVAL;

  const size_t need = round_up((size_t)bp_words(T, in.W, in.M) * 4, 256);
  const bool multi = geometry_is_multi(in.W, in.M);
  if (workspace && (ws_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u)))
    return CTCALIGN_EINVAL;
  const bool padded = !(C == in.stride && aligned16(emission));
  // the context's arena and pad buffer are shared across streams: wait for
  // the last call that used them, and let the next one wait for this one
  const bool shared = !workspace || padded;
  if (shared) {
    if (!ctx->arena_ev) HIP_TRY(hipEventCreateWithFlags(&ctx->arena_ev, hipEventDisableTiming));
    if (ctx->arena_used && ctx->arena_stream != st) HIP_TRY(hipStreamWaitEvent(st, ctx->arena_ev, 0));
  }
  char* ws;
  if (workspace) {
    ws = static_cast<char*>(workspace);
  } else {
    rc = ctx->ws.reserve(need);
    if (rc) return rc;
    ws = static_cast<char*>(ctx->ws.ptr);
  }
  in.bp = reinterpret_cast<uint32_t*>(ws);

  if (!padded) {
    in.em = emission;
  } else {
    // re-layout rows to the compiled stride in the context's pad buffer
    rc = ctx->pad.reserve((size_t)T * in.stride * sizeof(float));
    if (rc) return rc;
    const PadDesc pd{emission, static_cast<float*>(ctx->pad.ptr), T, C, in.stride, 0};
    HIP_TRY(launch_pad_one(pd, st));
    in.em = static_cast<float*>(ctx->pad.ptr);
  }
  CTCA_LOG(2, "align T=%d C=%d L=%d -> W=%d M=%d stride=%d", T, C, L, in.W, in.M, in.stride);
  if (multi) {
    rc = launch_multi_serial(ctx->device, in, st);
    if (rc) return rc;
  } else {
    HIP_TRY(launch_one(in, st));
  }
  if (shared) {
    HIP_TRY(hipEventRecord(ctx->arena_ev, st));
    ctx->arena_stream = st;
    ctx->arena_used = true;
  }
  return CTCALIGN_OK;
}

// ---- checkpointed long form ---------------------------------------------------

// Layout of a checkpointed alignment: the multi-workgroup layout with the
// fewest states per lane that holds S (W = 0 if none does: the regular path
// runs), K frames per stretch and the workspace parts.
struct CkPlan {
  Geo g{0, 0};
  int K = 0;
  int nstretch = 0;       // stretches of K frames (the last may be shorter)
  int64_t spad = 0;       // floats per column
  size_t off_cols = 0, off_bp = 0, bytes = 0;   // [state | columns | backpointers]
};

CkPlan ck_plan(int32_t T, int32_t L, int32_t K) {
  CkPlan p;
  const int S = 2 * L + 1;
  if (T > kXMaxT) return p;
  for (int M : kMenuMulti) {
    const int W = (S + kWave * M - 1) / (kWave * M);
    if (geometry_supported_ck(W, M) && geo_ok(S, W, M)) {
      p.g = Geo{W, M};
      break;
    }
  }
  if (p.g.W == 0) return p;
  if (K <= 0) {
    // about sqrt(T * 4 / (3/16)) minimises columns (4 bytes per state) plus
    // one stretch's backpointers (3/16 byte per state and frame); but each
    // stretch first fills the workgroup pipeline (a workgroup starts about
    // one 32-frame block after the one below it), so a stretch spans at
    // least four fills
    const int groups = (p.g.W + kXWaves - 1) / kXWaves;
    K = std::max((int)(4.6 * std::sqrt((double)T)), 4 * kBlk * groups);
  }
  K = std::max(kBlk, (K + kBlk - 1) / kBlk * kBlk);
  if ((int64_t)T <= (int64_t)K + 1) {   // one stretch: the regular path
    p.g = Geo{0, 0};
    return p;
  }
  p.K = K;
  p.nstretch = (T - 1 + K - 1) / K;
  p.spad = (int64_t)p.g.W * kWave * p.g.M;
  p.off_cols = 256;
  p.off_bp = p.off_cols + round_up((size_t)p.nstretch * (size_t)p.spad * sizeof(float), 256);
  p.bytes = p.off_bp + round_up((size_t)bp_words(K + 1, p.g.W, p.g.M) * 4, 256);
  return p;
}

uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

extern "C" {

const char* ctcalign_strerror(int status) {
  switch (status) {
    case CTCALIGN_OK: return "ok";
    case CTCALIGN_EINVAL: return "invalid argument or label";
    case CTCALIGN_EINFEASIBLE: return "no alignment with finite score";
    case CTCALIGN_ENOMEM: return "out of memory or over budget";
    case CTCALIGN_EDEVICE: return "HIP runtime error or device watchdog";
    case CTCALIGN_EAGAIN: return "queue full, try again";
    case CTCALIGN_EBUSY: return "not finished yet";
    default: return "unknown status";
  }
}

int ctcalign_version(void) { return 100; }

int ctcalign_tune_set(ctcalign_ctx* ctx, int32_t kind, int32_t s_lo, int32_t s_hi, int32_t C,
                      int32_t W, int32_t M) {
  if (!ctx || (kind != 0 && kind != 1) || s_lo < 1 || s_hi < s_lo || s_hi > kMaxS || C < 1 ||
      C > kMaxC)
    return CTCALIGN_EINVAL;
  if (W == 0) {
    ctx->tune.set_range(kind, s_lo, s_hi, C, Geo{0, 0});
    return CTCALIGN_OK;
  }
  const bool ok = kind == 0 ? geometry_supported_one(W, M) : geometry_supported_pack(W, M);
  if (!ok) return CTCALIGN_EINVAL;
  // the geometry must hold every S of the range (overrides are per 64-state bucket)
  const int lo = s_lo / kWave * kWave, hi = std::min<int64_t>(s_hi / kWave * kWave + kWave - 1, kMaxS);
  for (int S = std::max(lo, 1); S <= hi; ++S)
    if (S >= s_lo && S <= s_hi && !geo_ok(S, W, M)) return CTCALIGN_EINVAL;
  ctx->tune.set_range(kind, s_lo, s_hi, C, Geo{W, M});
  return CTCALIGN_OK;
}

int ctcalign_tune_get(ctcalign_ctx* ctx, int32_t kind, int32_t S, int32_t C, int32_t* W,
                      int32_t* M) {
  if (!ctx || !W || !M || S < 1 || S > kMaxS || C < 1 || C > kMaxC || (kind != 0 && kind != 1))
    return CTCALIGN_EINVAL;
  const Geo g = kind == 0 ? ctx->tune.pick_one(S, C) : ctx->tune.pick_pack(S, C, 0);
  *W = g.W;
  *M = g.M;
  return g.W > 0 ? CTCALIGN_OK : CTCALIGN_EINVAL;
}

int ctcalign_tune_knob(ctcalign_ctx* ctx, int32_t knob, double value, double* previous) {
  if (!ctx) return CTCALIGN_EINVAL;
  TuneTable& t = ctx->tune;
  switch (knob) {
    case CTCALIGN_KNOB_PACK_TARGET_M:
      if (previous) *previous = t.pack_target_m;
      if (value < 2 || value > 16) return CTCALIGN_EINVAL;
      t.pack_target_m = (int)value;
      return CTCALIGN_OK;
    case CTCALIGN_KNOB_CRIT_FRAC:
      if (previous) *previous = t.crit_frac;
      if (!(value >= 0.0 && value <= 1.0)) return CTCALIGN_EINVAL;
      t.crit_frac = value;
      return CTCALIGN_OK;
    case CTCALIGN_KNOB_CRIT_PER_CU:
      if (previous) *previous = t.crit_per_cu;
      if (!(value >= 0.0 && value <= 4.0)) return CTCALIGN_EINVAL;
      t.crit_per_cu = value;
      return CTCALIGN_OK;
    default:
      return CTCALIGN_EINVAL;
  }
}

int ctcalign_tune_save(ctcalign_ctx* ctx, const char* path) {
  if (!ctx || !path) return CTCALIGN_EINVAL;
  FILE* f = std::fopen(path, "w");
  if (!f) return CTCALIGN_EINVAL;
  std::fprintf(f, "# libctcalign tuning table v2: kind class bucket W M; knob id value\n");
  std::fprintf(f, "knob %d %d\n", (int)CTCALIGN_KNOB_PACK_TARGET_M, ctx->tune.pack_target_m);
  std::fprintf(f, "knob %d %.17g\n", (int)CTCALIGN_KNOB_CRIT_FRAC, ctx->tune.crit_frac);
  std::fprintf(f, "knob %d %.17g\n", (int)CTCALIGN_KNOB_CRIT_PER_CU, ctx->tune.crit_per_cu);
  for (int kind = 0; kind < 2; ++kind)
    for (int c = 0; c < 2; ++c) {
      const auto& t = kind == 0 ? ctx->tune.one_override[c] : ctx->tune.pack_override[c];
      for (size_t b = 0; b < t.size(); ++b)
        if (t[b].W > 0) std::fprintf(f, "%d %d %zu %d %d\n", kind, c, b, t[b].W, t[b].M);
    }
  std::fclose(f);
  return CTCALIGN_OK;
}

int ctcalign_tune_load(ctcalign_ctx* ctx, const char* path) {
  if (!ctx || !path) return CTCALIGN_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return CTCALIGN_EINVAL;
  char line[256];
  int rc = CTCALIGN_OK;
  while (std::fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    int knob;
    double kv;
    if (std::sscanf(line, "knob %d %lf", &knob, &kv) == 2) {
      if (ctcalign_tune_knob(ctx, knob, kv, nullptr) != CTCALIGN_OK) rc = CTCALIGN_EINVAL;
      continue;
    }
    int kind, c, b, W, M;
    if (std::sscanf(line, "%d %d %d %d %d", &kind, &c, &b, &W, &M) != 5) continue;
    if ((kind != 0 && kind != 1) || (c != 0 && c != 1) || b < 0 || b > kMaxS / kWave) {
      rc = CTCALIGN_EINVAL;
      continue;
    }
    const bool ok = kind == 0 ? geometry_supported_one(W, M) : geometry_supported_pack(W, M);
    if (!ok) {
      rc = CTCALIGN_EINVAL;
      continue;
    }
    // applied only where it holds the whole bucket; pick_* re-checks per S
    ctx->tune.set_range(kind, b * kWave, b * kWave + kWave - 1, c == 0 ? 32 : 256, Geo{W, M});
  }
  std::fclose(f);
  return rc;
}

int ctcalign_ctx_create(int device, ctcalign_ctx** out) {
  if (!out) return CTCALIGN_EINVAL;
  *out = nullptr;
  if (device < 0) HIP_TRY(hipGetDevice(&device));
  HIP_TRY(hipSetDevice(device));
  ctcalign_ctx* c = new (std::nothrow) ctcalign_ctx();
  if (!c) return CTCALIGN_ENOMEM;
  c->device = device;
  int rc = CTCALIGN_OK;
  hipDeviceProp_t prop;
  if ((rc = map_hip(hipGetDeviceProperties(&prop, device), "props")) ||
      (rc = map_hip(hipStreamCreate(&c->stream), "stream")) ||
      (rc = map_hip(hipHostMalloc((void**)&c->h_status, 16 * sizeof(int32_t)), "pinned")) ||
      (rc = map_hip(hipMalloc((void**)&c->d_status, 16 * sizeof(int32_t)), "status")) ||
      (rc = map_hip(hipMalloc((void**)&c->d_total, 16 * sizeof(float)), "total"))) {
    ctcalign_ctx_destroy(c);
    return rc;
  }
  c->num_cu = prop.multiProcessorCount;
  c->tune.load_default(c->num_cu);
  // the allocation-free entry point's scratch array: its address on this
  // device, looked up once (the device is current here)
  if (noalloc_setup(device) != CTCALIGN_OK) CTCA_LOG(1, "no scratch array on device %d", device);
  if (const char* tc = std::getenv("CTCALIGN_TUNE_CACHE")) {
    if (ctcalign_tune_load(c, tc) != CTCALIGN_OK) CTCA_LOG(1, "tuning cache %s not (fully) loaded", tc);
  }
  *out = c;
  return CTCALIGN_OK;
}

int ctcalign_ctx_destroy(ctcalign_ctx* c) {
  if (!c) return CTCALIGN_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->cached) ctcalign_plan_destroy(c->cached);
  c->ws.release();
  c->pad.release();
  if (c->arena_ev) (void)hipEventDestroy(c->arena_ev);
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->d_status) (void)hipFree(c->d_status);
  if (c->d_total) (void)hipFree(c->d_total);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  {
    std::lock_guard<std::mutex> lk(g_default_mu);
    for (auto& d : g_default)
      if (d == c) d = nullptr;
  }
  delete c;
  return CTCALIGN_OK;
}

size_t ctcalign_workspace_bytes(ctcalign_ctx* ctx, int32_t T, int32_t L, int32_t C) {
  if (!ctx || T < 1 || L < 0 || C < 1 || C > kMaxC || 2 * (int64_t)L + 1 > kMaxS) return 0;
  const Geo g = ctx->tune.pick_one(2 * L + 1, C);
  return round_up((size_t)bp_words(T, g.W, g.M) * 4, 256);
}

int ctcalign_align_ex(ctcalign_ctx* ctx, const float* emission, int32_t T, int32_t C,
                      const int32_t* labels, int32_t L, int32_t blank, int32_t* out_path,
                      float* out_scores, float* out_total, int32_t* out_status, void* workspace,
                      size_t ws_bytes, ctcalign_stream stream) {
  if (!ctx) return CTCALIGN_EINVAL;
  int rc = validate_one(emission, T, C, labels, L, blank, out_path, out_scores);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  return launch_single(ctx, emission, T, C, labels, L, blank, out_path, out_scores, out_total,
                       out_status, workspace, ws_bytes, st);
}

int ctcalign_align(const float* emission, int32_t T, int32_t C, const int32_t* labels, int32_t L,
                   int32_t blank, int32_t* out_path, float* out_scores) {
  int rc = validate_one(emission, T, C, labels, L, blank, out_path, out_scores);
  if (rc) return rc;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return CTCALIGN_EDEVICE;
  ctcalign_ctx* ctx;
  {
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default[dev]) {
      rc = ctcalign_ctx_create(dev, &g_default[dev]);
      if (rc) return rc;
    }
    ctx = g_default[dev];
  }
  rc = launch_single(ctx, emission, T, C, labels, L, blank, out_path, out_scores, ctx->d_total,
                     ctx->d_status, nullptr, 0, ctx->stream);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(ctx->h_status, ctx->d_status, sizeof(int32_t), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return ctx->h_status[0];
}

size_t ctcalign_checkpointed_workspace_bytes(ctcalign_ctx* ctx, int32_t T, int32_t L, int32_t C,
                                             int32_t K) {
  if (!ctx || T < 1 || L < 0 || C < 1 || C > kMaxC || 2 * (int64_t)L + 1 > kMaxS || K < 0) return 0;
  const CkPlan p = ck_plan(T, L, K);
  if (p.g.W == 0) return ctcalign_workspace_bytes(ctx, T, L, C);
  return p.bytes;
}

int ctcalign_align_checkpointed(ctcalign_ctx* ctx, const float* emission, int32_t T, int32_t C,
                                const int32_t* labels, int32_t L, int32_t blank, int32_t* out_path,
                                float* out_scores, float* out_total, int32_t* out_status, int32_t K,
                                void* workspace, size_t ws_bytes, ctcalign_stream stream) {
  if (!ctx || K < 0) return CTCALIGN_EINVAL;
  int rc = validate_one(emission, T, C, labels, L, blank, out_path, out_scores);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const CkPlan p = ck_plan(T, L, K);
  if (p.g.W == 0)   // no checkpointed layout, or a single stretch
    return launch_single(ctx, emission, T, C, labels, L, blank, out_path, out_scores, out_total,
                         out_status, workspace, ws_bytes, st);
  if (workspace && (ws_bytes < p.bytes || (reinterpret_cast<uintptr_t>(workspace) & 255u)))
    return CTCALIGN_EINVAL;
  const int stride = row_stride_for(C);
  const bool padded = !(C == stride && aligned16(emission));
  const bool shared = !workspace || padded;
  if (shared) {
    if (!ctx->arena_ev) HIP_TRY(hipEventCreateWithFlags(&ctx->arena_ev, hipEventDisableTiming));
    if (ctx->arena_used && ctx->arena_stream != st) HIP_TRY(hipStreamWaitEvent(st, ctx->arena_ev, 0));
  }
  char* ws;
  if (workspace) {
    ws = static_cast<char*>(workspace);
  } else {
    rc = ctx->ws.reserve(p.bytes);
    if (rc) return rc;
    ws = static_cast<char*>(ctx->ws.ptr);
  }
  const float* em = emission;
  if (padded) {
    rc = ctx->pad.reserve((size_t)T * stride * sizeof(float));
    if (rc) return rc;
    const PadDesc pd{emission, static_cast<float*>(ctx->pad.ptr), T, C, stride, 0};
    HIP_TRY(launch_pad_one(pd, st));
    em = static_cast<float*>(ctx->pad.ptr);
  }
  CkArgs ck{};
  ck.ck = reinterpret_cast<float*>(ws + p.off_cols);
  ck.state = reinterpret_cast<int32_t*>(ws);
  ck.spad = (int32_t)p.spad;
  ck.every = p.K;
  Inst in{};
  in.C = C;
  in.L = L;
  in.blank = blank;
  in.lab = labels;
  in.stride = stride;
  in.W = p.g.W;
  in.M = p.g.M;
  in.prio = 0;
  // first pass: the whole alignment, columns only
  in.T = T;
  in.em = em;
  in.path = out_path;
  in.scores = out_scores;
  in.total = out_total;
  in.status = out_status;
  in.bp = reinterpret_cast<uint32_t*>(ws + p.off_bp);   // not written in this pass
  CTCA_LOG(2, "align_checkpointed T=%d C=%d L=%d -> W=%d M=%d K=%d stretches=%d bytes=%zu", T, C, L,
           in.W, in.M, p.K, p.nstretch, p.bytes);
  rc = launch_multi_serial(ctx->device, in, st, &ck, kModeCkFirst);
  if (rc) return rc;
  // stretches, last first: stretch k covers frames kK .. min(kK + K, T - 1)
  in.total = nullptr;
  for (int k = p.nstretch - 1; k >= 0; --k) {
    const int t0 = k * p.K;
    const int Tk = std::min(p.K, T - 1 - t0) + 1;
    in.T = Tk;
    in.em = em + (int64_t)t0 * stride;
    in.path = out_path + t0;
    in.scores = out_scores + t0;
    ck.col = k;
    rc = launch_multi_serial(ctx->device, in, st, &ck, kModeCkSeg);
    if (rc) return rc;
  }
  if (shared) {
    HIP_TRY(hipEventRecord(ctx->arena_ev, st));
    ctx->arena_stream = st;
    ctx->arena_used = true;
  }
  return CTCALIGN_OK;
}

int ctcalign_token_spans(const int32_t* path, const float* scores, int32_t T, int32_t blank,
                         int32_t max_spans, int32_t* out_token, int32_t* out_start,
                         int32_t* out_end, float* out_score, int32_t* out_count,
                         ctcalign_stream stream) {
  if (!path || !scores || !out_count || T < 1 || T > (1 << 30) || max_spans < 0 || blank < 0 ||
      (max_spans > 0 && (!out_token || !out_start || !out_end || !out_score)))
    return CTCALIGN_EINVAL;
  HIP_TRY(launch_spans(path, scores, T, blank, max_spans, out_token, out_start, out_end, out_score,
                       out_count, static_cast<hipStream_t>(stream)));
  return CTCALIGN_OK;
}

// ---- batched plans -----------------------------------------------------------

int ctcalign_plan_create(ctcalign_ctx* ctx, int32_t N, const float* emissions,
                         const int64_t* em_off, const int32_t* T, const int32_t* C,
                         const int32_t* labels, const int64_t* lab_off, const int32_t* L,
                         int32_t blank, int32_t* out_paths, float* out_scores,
                         const int64_t* frame_off, float* out_totals, int32_t* out_status,
                         ctcalign_plan** plan_out) {
  if (!ctx || !plan_out || N < 0) return CTCALIGN_EINVAL;
  *plan_out = nullptr;
  if (N > 0 && (!emissions || !em_off || !T || !C || !lab_off || !L || !out_paths ||
                !out_scores || !frame_off || !out_totals || !out_status))
    return CTCALIGN_EINVAL;
  for (int i = 0; i < N; ++i) {
    if (T[i] < 1 || T[i] > (1 << 30) || C[i] < 1 || C[i] > kMaxC || L[i] < 0 || blank < 0 ||
        blank >= C[i] || em_off[i] < 0 || lab_off[i] < 0 || frame_off[i] < 0)
      return CTCALIGN_EINVAL;
    if (L[i] > 0 && !labels) return CTCALIGN_EINVAL;
    if (2 * (int64_t)L[i] + 1 > kMaxS) return CTCALIGN_EINVAL;
  }
  HIP_TRY(hipSetDevice(ctx->device));

  ctcalign_plan* p = new (std::nothrow) ctcalign_plan();
  if (!p) return CTCALIGN_ENOMEM;
  p->ctx = ctx;
  p->n = N;

  std::vector<Inst> insts(N);
  std::vector<PadDesc> pads;
  std::vector<double> cost(N);
  size_t bp_total = 0, pad_total = 0;
  std::vector<size_t> bp_off(N), pad_off(N, SIZE_MAX);
  std::vector<char> is_long(N, 0);
  for (int i = 0; i < N; ++i) {
    Inst& in = insts[i];
    in.T = T[i];
    in.C = C[i];
    in.L = L[i];
    in.blank = blank;
    in.lab = labels ? labels + lab_off[i] : nullptr;
    in.path = out_paths + frame_off[i];
    in.scores = out_scores + frame_off[i];
    in.total = out_totals + i;
    in.status = out_status + i;
    in.stride = row_stride_for(C[i]);
    const int S = 2 * L[i] + 1;
    const bool big = S > ctx->tune.max_pack_states();
    const Geo g = big ? ctx->tune.pick_long(S) : ctx->tune.pick_pack(S, C[i], T[i]);
    const bool supported = big ? geometry_supported_long_batch(g.W, g.M) : geometry_supported_pack(g.W, g.M);
    if (!supported || !geo_ok(S, g.W, g.M)) {
      delete p;
      return CTCALIGN_EINVAL;   // no compiled layout holds this trellis
    }
    is_long[i] = big;
    in.W = g.W;
    in.M = g.M;
    in.prio = 0;
    cost[i] = (double)T[i] * ctx->tune.step_cost(g, in.stride);
    const float* src = emissions + em_off[i];
    if (C[i] != in.stride || !aligned16(src)) {
      pad_off[i] = pad_total;
      pad_total += round_up((size_t)T[i] * in.stride * sizeof(float), 256);
    }
  }

  // The batch's longest chains bound the whole pass: the ones whose chain
  // (frames x per-frame latency of their pack layout) is close to the longest
  // run in 8-wave workgroups with fewer states per lane instead.
  std::vector<char> is_crit(N, 0);
  std::vector<int> crit_order;
  {
    std::vector<int> cand;
    double top = 0;
    for (int i = 0; i < N; ++i)
      if (!is_long[i]) top = std::max(top, ctx->tune.chain_ns(insts[i]));
    for (int i = 0; i < N; ++i)
      if (!is_long[i] && top > 0 && ctx->tune.chain_ns(insts[i]) >= ctx->tune.crit_frac * top) cand.push_back(i);
    std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) {
      return ctx->tune.chain_ns(insts[a]) > ctx->tune.chain_ns(insts[b]);
    });
    if ((int)cand.size() > ctx->tune.crit_max()) cand.resize(ctx->tune.crit_max());
    for (int i : cand) {
      const Geo g = ctx->tune.pick_crit(2 * insts[i].L + 1);
      if (g.W == 0 || !geometry_supported_crit(g.W, g.M) || g.M >= insts[i].M) continue;
      insts[i].W = g.W;
      insts[i].M = g.M;
      insts[i].prio = 3;         // issue priority over the packs sharing its CU
      is_crit[i] = 1;
      crit_order.push_back(i);   // longest chain first
    }
  }
  for (int i = 0; i < N; ++i) {
    bp_off[i] = bp_total;
    bp_total += round_up((size_t)bp_words(T[i], insts[i].W, insts[i].M) * 4, 256);
  }

  // LPT order: most expensive first
  std::vector<int> order(N);
  for (int i = 0; i < N; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });

  // packs of kPackWaves waves: kPackWaves / W alignments of W waves each,
  // neighbours in cost order, so a pack's waves finish at similar times
  std::vector<Pack> packs;
  std::vector<double> pack_cost;
  auto blank_pack = [] {
    Pack pk;
    for (int k = 0; k < kPackWaves; ++k) {
      pk.inst[k] = -1;
      pk.seg[k] = 0;
      pk.first[k] = (int16_t)k;
    }
    return pk;
  };
  Pack open[kPackWaves + 1];
  int nopen[kPackWaves + 1] = {};
  double copen[kPackWaves + 1] = {};
  for (int W = 1; W <= kPackWaves; ++W) open[W] = blank_pack();
  std::vector<int> long_order;
  for (int idx : order) {
    if (is_crit[idx]) continue;
    if (is_long[idx]) {
      long_order.push_back(idx);   // already longest first
      continue;
    }
    const int W = insts[idx].W;    // 1, 2, 4 or 8 (geometry_supported_pack)
    const int m = nopen[W];
    for (int k = 0; k < W; ++k) {
      open[W].inst[m * W + k] = idx;
      open[W].seg[m * W + k] = (int16_t)k;
      open[W].first[m * W + k] = (int16_t)(m * W);
    }
    copen[W] = std::max(copen[W], cost[idx]);
    if (++nopen[W] == kPackWaves / W) {
      packs.push_back(open[W]);
      pack_cost.push_back(copen[W]);
      open[W] = blank_pack();
      nopen[W] = 0;
      copen[W] = 0;
    }
  }
  for (int W = 1; W <= kPackWaves; ++W)
    if (nopen[W]) {
      packs.push_back(open[W]);
      pack_cost.push_back(copen[W]);
    }
  {
    std::vector<int> po(packs.size());
    for (size_t i = 0; i < po.size(); ++i) po[i] = (int)i;
    std::stable_sort(po.begin(), po.end(), [&](int a, int b) { return pack_cost[a] > pack_cost[b]; });
    std::vector<Pack> sorted(packs.size());
    std::vector<double> sorted_cost(packs.size());
    for (size_t i = 0; i < po.size(); ++i) {
      sorted[i] = packs[po[i]];
      sorted_cost[i] = pack_cost[po[i]];
    }
    packs.swap(sorted);
    pack_cost.swap(sorted_cost);
  }
  p->npacks = (int)packs.size();
  if (!std::getenv("CTCALIGN_NO_PRIO")) ctx->tune.assign_priorities(insts, packs, pack_cost);

  int rc = CTCALIGN_OK;
  auto fail = [&](int code) {
    ctcalign_plan_destroy(p);
    return code;
  };
  p->bp_bytes = std::max(bp_total, (size_t)256);
  if ((rc = map_hip(hipMalloc(&p->d_bp, p->bp_bytes), "bp"))) return fail(rc);
  if (pad_total && (rc = map_hip(hipMalloc(&p->d_padbuf, pad_total), "padbuf"))) return fail(rc);
  for (int i = 0; i < N; ++i) {
    Inst& in = insts[i];
    in.bp = reinterpret_cast<uint32_t*>(static_cast<char*>(p->d_bp) + bp_off[i]);
    const float* src = emissions + em_off[i];
    if (pad_off[i] != SIZE_MAX) {
      float* dst = reinterpret_cast<float*>(static_cast<char*>(p->d_padbuf) + pad_off[i]);
      pads.push_back(PadDesc{src, dst, in.T, in.C, in.stride, 0});
      p->pad_max = std::max(p->pad_max, (int64_t)in.T * in.stride);
      in.em = dst;
    } else {
      in.em = src;
    }
  }
  p->npad = (int)pads.size();
  p->nlong = (int)long_order.size();
  p->ncrit = (int)crit_order.size();
  if (p->ncrit &&
      ((rc = map_hip(hipMalloc((void**)&p->d_crit, sizeof(int) * (p->ncrit + 1)), "crit")) ||
       (rc = map_hip(hipMemcpy(p->d_crit, crit_order.data(), sizeof(int) * p->ncrit,
                               hipMemcpyHostToDevice), "h2d"))))
    return fail(rc);
  if (p->nlong &&
      ((rc = map_hip(hipMalloc((void**)&p->d_order, sizeof(int) * p->nlong), "order")) ||
       (rc = map_hip(hipMemcpy(p->d_order, long_order.data(), sizeof(int) * p->nlong,
                               hipMemcpyHostToDevice), "h2d")) ||
       (rc = map_hip(hipMalloc((void**)&p->d_head_long, sizeof(int)), "head"))))
    return fail(rc);
  if ((rc = map_hip(hipMalloc((void**)&p->d_insts, sizeof(Inst) * std::max(N, 1)), "insts")) ||
      (rc = map_hip(hipMalloc((void**)&p->d_packs, sizeof(Pack) * std::max(p->npacks, 1)), "packs")) ||
      (rc = map_hip(hipMalloc((void**)&p->d_head, sizeof(int)), "head")))
    return fail(rc);
  if (p->npad && (rc = map_hip(hipMalloc((void**)&p->d_pad, sizeof(PadDesc) * p->npad), "pad")))
    return fail(rc);
  if (N && (rc = map_hip(hipMemcpy(p->d_insts, insts.data(), sizeof(Inst) * N, hipMemcpyHostToDevice), "h2d")))
    return fail(rc);
  if (p->npacks && (rc = map_hip(hipMemcpy(p->d_packs, packs.data(), sizeof(Pack) * p->npacks,
                                           hipMemcpyHostToDevice), "h2d")))
    return fail(rc);
  if (p->npad && (rc = map_hip(hipMemcpy(p->d_pad, pads.data(), sizeof(PadDesc) * p->npad,
                                         hipMemcpyHostToDevice), "h2d")))
    return fail(rc);

  // Oversubscribed on purpose: workgroups never wait for each other, so the
  // ones that do not fit yet start when a resident one leaves, find the queue
  // drained and exit; the hardware fills every CU to its real occupancy.
  p->grid = std::min(p->npacks, ctx->num_cu * 16);
  if (const char* tr = std::getenv("CTCALIGN_TRACE")) {
    if (std::atoi(tr) > 0 && p->npacks &&
        (rc = map_hip(hipMalloc((void**)&p->d_trace, sizeof(int64_t) * 3 * p->npacks), "trace")))
      return fail(rc);
  }
  if (p->grid < 1) p->grid = 1;

  // capture: [pad] -> queue reset -> persistent kernel
  if ((rc = map_hip(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "capstream")))
    return fail(rc);
  if ((rc = map_hip(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "capture")))
    return fail(rc);
  hipError_t e = hipSuccess;
  if (p->npad) e = launch_pad(p->d_pad, p->npad, p->pad_max, p->cap_stream);
  // the longest chains on a parallel branch, launched first
  if (e == hipSuccess && p->ncrit) {
    if ((e = hipStreamCreateWithFlags(&p->crit_stream, hipStreamNonBlocking)) == hipSuccess &&
        (e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming)) == hipSuccess &&
        (e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming)) == hipSuccess &&
        (e = hipEventRecord(p->ev_fork, p->cap_stream)) == hipSuccess &&
        (e = hipStreamWaitEvent(p->crit_stream, p->ev_fork, 0)) == hipSuccess &&
        (e = launch_persistent_crit(p->d_insts, p->d_crit, p->ncrit, p->crit_stream)) == hipSuccess)
      e = hipEventRecord(p->ev_join, p->crit_stream);
  }
  if (e == hipSuccess) e = launch_fill(p->d_head, 1, 0, p->cap_stream);
  if (e == hipSuccess && p->npacks)
    e = launch_persistent(p->d_insts, p->d_packs, p->npacks, p->d_head, p->grid, p->cap_stream,
                          p->d_trace);
  if (e == hipSuccess && p->nlong) e = launch_fill(p->d_head_long, 1, 0, p->cap_stream);
  if (e == hipSuccess && p->nlong)
    e = launch_persistent_long(p->d_insts, p->d_order, p->nlong, p->d_head_long,
                               std::min(p->nlong, ctx->num_cu * 4), p->cap_stream);
  if (e == hipSuccess && p->ncrit) e = hipStreamWaitEvent(p->cap_stream, p->ev_join, 0);
  hipError_t e2 = hipStreamEndCapture(p->cap_stream, &p->graph);
  if (e != hipSuccess) return fail(map_hip(e, "captured launch"));
  if ((rc = map_hip(e2, "end capture"))) return fail(rc);
  if ((rc = map_hip(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "instantiate")))
    return fail(rc);
  CTCA_LOG(2, "plan: N=%d packs=%d grid=%d bp=%zu pad=%zu", N, p->npacks, p->grid, bp_total, pad_total);
  *plan_out = p;
  return CTCALIGN_OK;
}

int ctcalign_plan_run(ctcalign_plan* p, ctcalign_stream stream) {
  if (!p) return CTCALIGN_EINVAL;
  HIP_TRY(hipSetDevice(p->ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!p->run_ev) HIP_TRY(hipEventCreateWithFlags(&p->run_ev, hipEventDisableTiming));
  if (p->ran && p->run_stream != st) HIP_TRY(hipStreamWaitEvent(st, p->run_ev, 0));
  HIP_TRY(hipGraphLaunch(p->exec, st));
  HIP_TRY(hipEventRecord(p->run_ev, st));
  p->run_stream = st;
  p->ran = true;
  return CTCALIGN_OK;
}

int ctcalign_plan_trace(ctcalign_plan* p, int32_t max_packs, int64_t* out_times,
                        int32_t* out_insts, int32_t* npacks) {
  if (!p || !npacks) return CTCALIGN_EINVAL;
  *npacks = p->npacks;
  if (!p->d_trace) return CTCALIGN_EINVAL;
  const int n = std::min(max_packs, p->npacks);
  if (out_times) HIP_TRY(hipMemcpy(out_times, p->d_trace, sizeof(int64_t) * 3 * n, hipMemcpyDeviceToHost));
  if (out_insts) {
    std::vector<Pack> pk(n);
    HIP_TRY(hipMemcpy(pk.data(), p->d_packs, sizeof(Pack) * n, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < kPackWaves; ++k) out_insts[kPackWaves * i + k] = pk[i].inst[k];
  }
  return CTCALIGN_OK;
}

int ctcalign_plan_destroy(ctcalign_plan* p) {
  if (!p) return CTCALIGN_OK;
  (void)hipSetDevice(p->ctx->device);
  (void)hipDeviceSynchronize();
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->d_insts) (void)hipFree(p->d_insts);
  if (p->d_packs) (void)hipFree(p->d_packs);
  if (p->d_pad) (void)hipFree(p->d_pad);
  if (p->d_head) (void)hipFree(p->d_head);
  if (p->d_bp) (void)hipFree(p->d_bp);
  if (p->d_padbuf) (void)hipFree(p->d_padbuf);
  if (p->d_trace) (void)hipFree(p->d_trace);
  if (p->d_order) (void)hipFree(p->d_order);
  if (p->d_head_long) (void)hipFree(p->d_head_long);
  if (p->d_crit) (void)hipFree(p->d_crit);
  if (p->crit_stream) (void)hipStreamDestroy(p->crit_stream);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->run_ev) (void)hipEventDestroy(p->run_ev);
  if (p->ctx && p->ctx->cached == p) p->ctx->cached = nullptr;
  delete p;
  return CTCALIGN_OK;
}

int ctcalign_align_batched(ctcalign_ctx* ctx, int32_t N, const float* emissions,
                           const int64_t* em_off, const int32_t* T, const int32_t* C,
                           const int32_t* labels, const int64_t* lab_off, const int32_t* L,
                           int32_t blank, int32_t* out_paths, float* out_scores,
                           const int64_t* frame_off, float* out_totals, int32_t* out_status,
                           ctcalign_stream stream) {
  if (!ctx || N < 0) return CTCALIGN_EINVAL;
  if (N > 0 && (!em_off || !T || !C || !lab_off || !L || !frame_off)) return CTCALIGN_EINVAL;
  uint64_t h = 1469598103934665603ull;
  const void* ptrs[] = {emissions, labels, out_paths, out_scores, out_totals, out_status};
  h = fnv(h, ptrs, sizeof(ptrs));
  h = fnv(h, &N, sizeof(N));
  h = fnv(h, &blank, sizeof(blank));
  if (N > 0) {
    h = fnv(h, em_off, sizeof(int64_t) * N);
    h = fnv(h, T, sizeof(int32_t) * N);
    h = fnv(h, C, sizeof(int32_t) * N);
    h = fnv(h, lab_off, sizeof(int64_t) * N);
    h = fnv(h, L, sizeof(int32_t) * N);
    h = fnv(h, frame_off, sizeof(int64_t) * N);
  }
  if (!ctx->cached || ctx->cached_key != h) {
    if (ctx->cached) ctcalign_plan_destroy(ctx->cached);
    ctcalign_plan* p = nullptr;
    int rc = ctcalign_plan_create(ctx, N, emissions, em_off, T, C, labels, lab_off, L, blank,
                                  out_paths, out_scores, frame_off, out_totals, out_status, &p);
    if (rc) return rc;
    ctx->cached = p;
    ctx->cached_key = h;
  }
  return ctcalign_plan_run(ctx->cached, stream);
}

}  // extern "C"
