/*
 * libctcalign -- CTC forced alignment on AMD Instinct MI355X (gfx950).
 *
 * Operation (paper Sec. 4, paragraph "CTC-based forced alignment"): given
 * per-frame log-probabilities emission[T][C] of a CTC-trained model and a
 * transcript labels[L] (class ids, none equal to the blank), find the
 * frame-level alignment of highest total log-probability among all CTC
 * alignments of the transcript (all frame labellings that collapse to it when
 * runs are merged and blanks dropped).  This is the Viterbi maximum over the
 * blank-interleaved trellis of S = 2L+1 states:
 *
 *   y'_s = blank (s even), labels[(s-1)/2] (s odd)
 *   a_0(s) = emission[0][y'_s] for s in {0,1}, -inf otherwise
 *   a_t(s) = emission[t][y'_s] + max(a_{t-1}(s), a_{t-1}(s-1),
 *                                     a_{t-1}(s-2) if s odd, s>=3, y'_s != y'_{s-2})
 *   end state S-1 or S-2 (0 when L = 0), then backtrack.
 *
 * Exactness contract: every result is bitwise identical to a plain
 * sequential float32 evaluation of the recurrence above with one IEEE add
 * (round to nearest even, denormals kept) per state and frame, the tie rule
 * "prefer s, then s-1, then s-2" (first maximum under strict '>'), and the
 * end-state tie resolved to S-1.
 *
 * Outputs per utterance:
 *   out_path[t]   int32  the class id y'_{s_t} aligned to frame t (blanks included)
 *   out_scores[t] float  emission[t][out_path[t]]
 *   total         float  a_{T-1}(end state): the alignment's log-probability,
 *                        equal bitwise to the float32 left fold of out_scores
 *
 * Memory: unless stated otherwise every data pointer is a DEVICE pointer
 * (hipMalloc'd or a torch tensor's data_ptr()) on the context's device; the
 * caller owns all inputs, outputs and workspaces; the library never frees
 * or keeps them after the call returns (asynchronous calls: until the
 * stream reaches the work).  Outputs must not overlap inputs.
 * Layouts: emission row-major [T][C] float32, row stride C; labels int32.
 * Limits: 1 <= T <= 2^30, 1 <= C <= 256, 0 <= L, T*(2L+1) < 2^62.
 *
 * Errors: every function returns a status (CTCALIGN_OK = 0 on success) and
 * never aborts.  Argument errors found on the host return CTCALIGN_EINVAL
 * before any device work and leave outputs untouched.  Per-utterance
 * conditions found on the device are reported through the status outputs:
 *   EINVAL      a label outside [0, C) or equal to the blank: path = -1,
 *               scores = NaN, total = NaN
 *   EINFEASIBLE no alignment with finite score (e.g. T < L + repeats):
 *               path = -1, scores = -inf, total = -inf
 * HIP runtime failures map to CTCALIGN_EDEVICE.
 *
 * Threads: a context may be used by one host thread at a time.
 */
#ifndef CTCALIGN_H_
#define CTCALIGN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CTCALIGN_OK = 0,
  CTCALIGN_EINVAL = 1,      /* invalid argument or label */
  CTCALIGN_EINFEASIBLE = 2, /* no alignment with finite score */
  CTCALIGN_ENOMEM = 3,      /* allocation failed or over the memory budget */
  CTCALIGN_EDEVICE = 4,     /* HIP runtime error or device-side watchdog */
  CTCALIGN_EAGAIN = 5,      /* server queue full (non-blocking submit) */
  CTCALIGN_EBUSY = 6        /* request not finished yet (poll) */
};

typedef struct ctcalign_ctx ctcalign_ctx;
typedef struct ctcalign_plan ctcalign_plan;
typedef struct ctcalign_server ctcalign_server;
typedef void *ctcalign_stream; /* a hipStream_t; NULL = HIP's default (null) stream */

/* Human-readable name of a status code (static string, never NULL). */
const char *ctcalign_strerror(int status);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int ctcalign_version(void);

/* ---- contexts ----------------------------------------------------------- */

/* Creates a context on HIP device `device` (or the current device if < 0):
 * a stream, a cached workspace arena and the tuning table.  *ctx receives
 * the handle.  Errors: EINVAL (ctx NULL), EDEVICE. */
int ctcalign_ctx_create(int device, ctcalign_ctx **ctx);

/* Waits for the context's stream, frees everything it owns.  NULL is a no-op. */
int ctcalign_ctx_destroy(ctcalign_ctx *ctx);

/* Bytes of backpointer workspace one alignment of shape (T, L, C) needs under
 * the geometry this context would pick; 0 on invalid shape.  The backtrack of
 * the Viterbi recursion (paper Sec. 4, "CTC-based forced alignment") needs
 * the choice made at every state and frame: one bit per state and frame
 * here (a label state's choice between the two states below it is the bit of
 * the blank state under it), laid out per wavefront in whole 32-frame blocks,
 * so the size depends on the geometry (W, M)
 * and therefore on the context's tuning table and on C, not on (T, L) alone.
 * Query again after ctcalign_tune_set / _load. */
size_t ctcalign_workspace_bytes(ctcalign_ctx *ctx, int32_t T, int32_t L, int32_t C);

/* ---- geometry tuning ------------------------------------------------------
 * An alignment of S = 2L+1 states runs on W wavefronts with M states per lane
 * (W*64*M >= S).  kind 0 = single launches, kind 1 = the batched persistent
 * kernel.  The context's table maps (64-state bucket of S, class of C: C <= 32
 * or larger) to (W, M); empty buckets use the built-in cost model.  The
 * autotuner (paper_2310_17864_amd/tune.py) times candidates and fills it. */

/* Sets (W, M) for every S in [s_lo, s_hi] of C's class; W = 0 clears the
 * range.  EINVAL if the kernels do not compile that geometry or it cannot
 * hold some S of the range. */
int ctcalign_tune_set(ctcalign_ctx *ctx, int32_t kind, int32_t s_lo, int32_t s_hi, int32_t C,
                      int32_t W, int32_t M);

/* The geometry the context picks for (S, C). */
int ctcalign_tune_get(ctcalign_ctx *ctx, int32_t kind, int32_t S, int32_t C, int32_t *W,
                      int32_t *M);

/* Scheduling knobs of the batched plan, tuned on a whole workload
 * (paper_2310_17864_amd/tune.py --workload):
 *   PACK_TARGET_M  states per lane the pack kernel aims for (2..16; more
 *                  states per lane: fewer waves, longer frames)
 *   CRIT_FRAC      alignments whose modelled chain time is within this
 *                  fraction of the longest run as critical chains on their
 *                  own 8-wave workgroups (0 disables; 0..1)
 *   CRIT_PER_CU    at most this many critical chains per compute unit (0..4)
 * Plans created afterwards use the new value; *previous (nullable) receives
 * the old one.  EINVAL for an unknown knob or a value out of range. */
enum {
  CTCALIGN_KNOB_PACK_TARGET_M = 1,
  CTCALIGN_KNOB_CRIT_FRAC = 2,
  CTCALIGN_KNOB_CRIT_PER_CU = 3
};
int ctcalign_tune_knob(ctcalign_ctx *ctx, int32_t knob, double value, double *previous);

/* Writes / reads the table as text lines "kind class bucket W M" and
 * "knob id value" (host file path).  ctcalign_ctx_create loads
 * $CTCALIGN_TUNE_CACHE when it is set.  Entries the kernels cannot run are
 * skipped (EINVAL is returned). */
int ctcalign_tune_save(ctcalign_ctx *ctx, const char *path);
int ctcalign_tune_load(ctcalign_ctx *ctx, const char *path);

/* ---- one utterance ------------------------------------------------------ */

/* Forced alignment of one utterance (paper Sec. 4, "CTC-based forced
 * alignment": the frame-level alignment of a transcript to a CTC model's
 * outputs; the recurrence above).  Runs on the default context (created on
 * first use on the current device) and its stream, and waits for the result.
 * Returns OK, EINVAL, EINFEASIBLE (device-side outcome), ENOMEM or EDEVICE. */
int ctcalign_align(const float *emission, int32_t T, int32_t C,
                   const int32_t *labels, int32_t L, int32_t blank,
                   int32_t *out_path, float *out_scores);

/* The same alignment (paper Sec. 4, "CTC-based forced alignment"),
 * asynchronous on `stream` (NULL: HIP's null stream).
 * out_total (device, 1 float) and out_status (device, 1 int32) may be NULL.
 * workspace (device, >= ctcalign_workspace_bytes, 256-byte aligned) may be
 * NULL: the context's arena is used.  Calls that use the context's arena, or
 * its buffer for re-laid-out emission rows (C not 32 or 256, or a pointer
 * not 16-byte aligned), are ordered after the previous such call even when
 * they come on different streams (the stream waits for an event the last
 * one recorded).  Returns OK when the launch was queued; the alignment's own
 * status is written to *out_status.
 * Trellises above 4096 states run over several workgroups that exchange
 * boundary values through a per-device sync region: such launches are
 * cooperative, are serialised with each other across streams by an event
 * (so they cannot be captured into a HIP graph), and fail with EDEVICE if
 * the workgroups cannot all be resident. */
int ctcalign_align_ex(ctcalign_ctx *ctx, const float *emission, int32_t T, int32_t C,
                      const int32_t *labels, int32_t L, int32_t blank,
                      int32_t *out_path, float *out_scores, float *out_total,
                      int32_t *out_status, void *workspace, size_t ws_bytes,
                      ctcalign_stream stream);

/* Memory-bounded forced alignment of one long utterance: the same
 * alignment (paper Sec. 4, "CTC-based forced alignment", whose GPU path the
 * paper presents for long audio files), bitwise the same results as
 * ctcalign_align_ex, with a workspace that grows like sqrt(T) instead of T.
 * A first pass runs the recursion over all frames and keeps only the column
 * a_t of every K-th frame (4 bytes per state); then each stretch of K frames,
 * last first, is run again from its column with backpointers for those K
 * frames only, and backtracked from the state where the stretch after it
 * began.  Workspace: about (T/K) * S * 4 + K * S * 3/16 bytes
 * (ctcalign_checkpointed_workspace_bytes); the forward recursion runs twice.
 * K: frames per stretch, rounded up to a multiple of 32; 0 picks the
 * larger of about 4.6 * sqrt(T), which minimises the workspace, and four
 * times the pipeline fill of a stretch (32 frames per workgroup of eight
 * wavefronts), which keeps the second pass within a small factor of the
 * first.  Runs in the
 * multi-workgroup layout (513 <= S <= 32768, T < 2^21 - 64); other shapes,
 * and T <= K + 1, take the regular path of ctcalign_align_ex, whose
 * workspace ctcalign_checkpointed_workspace_bytes then reports.  Launches
 * are ordered on `stream` and serialised with other multi-workgroup launches
 * as described for ctcalign_align_ex.  Errors as ctcalign_align_ex; EINVAL
 * also for K < 0 or a workspace smaller than required. */
int ctcalign_align_checkpointed(ctcalign_ctx *ctx, const float *emission, int32_t T, int32_t C,
                                const int32_t *labels, int32_t L, int32_t blank,
                                int32_t *out_path, float *out_scores, float *out_total,
                                int32_t *out_status, int32_t K, void *workspace, size_t ws_bytes,
                                ctcalign_stream stream);

/* Workspace bytes of ctcalign_align_checkpointed for (T, L, C, K); 0 on an
 * invalid shape. */
size_t ctcalign_checkpointed_workspace_bytes(ctcalign_ctx *ctx, int32_t T, int32_t L, int32_t C,
                                             int32_t K);

/* For callers that cannot allocate device memory (work recorded under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * alignment of ctcalign_align_ex, bitwise the same results, asynchronous on
 * `stream`, with no allocation of any kind during the call.  Backpointers
 * and re-laid-out emission rows live in a fixed scratch array in device
 * memory, ctcalign_noalloc_scratch_bytes() = 64 MiB, one per device for the
 * life of the process (its address is looked up when a context is created on
 * the device).  Every call on one device shares that array: calls that
 * overlap in time on one device race and must be ordered by the caller (one
 * stream, or events).  Alignments run on one workgroup (S <= 32768): the
 * backpointers take about T * S * 3/16 bytes (plus T * 32 or T * 256 floats
 * when C is not 32 or 256, or the emission is not 16-byte aligned).
 * Errors: EINVAL as ctcalign_align_ex; ENOMEM when the call needs more
 * scratch than the array holds (nothing is launched); EDEVICE if the
 * context's device has no scratch address. */
int ctcalign_align_noalloc(ctcalign_ctx *ctx, const float *emission, int32_t T, int32_t C,
                           const int32_t *labels, int32_t L, int32_t blank,
                           int32_t *out_path, float *out_scores, float *out_total,
                           int32_t *out_status, ctcalign_stream stream);

/* Size in bytes of the per-device scratch array of ctcalign_align_noalloc. */
size_t ctcalign_noalloc_scratch_bytes(void);

/* Token spans of an alignment: the frame-level path (paper Sec. 4,
 * "CTC-based forced alignment") grouped into one segment per transcript
 * token, the step that turns a frame alignment into token time stamps for
 * segmentation (the method the paper cites there, Kuerzinger et al. 2020,
 * CTC segmentation).  Device pointers; asynchronous on `stream`:
 * each maximal run of frames with the same non-blank class is one span --
 * one per transcript token, since equal neighbouring tokens are separated by
 * a blank in any CTC alignment.  For span i (in frame order): out_token[i]
 * the class, out_start[i] / out_end[i] its first frame and one past its last,
 * out_score[i] the float32 left fold of its per-frame scores.  At most
 * max_spans spans are written; *out_count (device) receives the number found.
 * A failed alignment (path = -1) has no spans. */
int ctcalign_token_spans(const int32_t *path, const float *scores, int32_t T, int32_t blank,
                         int32_t max_spans, int32_t *out_token, int32_t *out_start,
                         int32_t *out_end, float *out_score, int32_t *out_count,
                         ctcalign_stream stream);

/* ---- many utterances: one persistent kernel over a device work queue ---- */

/* Builds a plan that aligns N utterances, each exactly as ctcalign_align_ex
 * would (paper Sec. 4, "CTC-based forced alignment"; the paper describes no
 * batching, this is a throughput layout of the same computation), packed in
 * flat device arrays.  Host arrays
 * (length N): em_off (element offset of each [T_i][C_i] emission in
 * `emissions`), T, C, lab_off (element offset in `labels`), L, frame_off
 * (element offset of each utterance's T_i outputs in out_paths/out_scores).
 * out_totals and out_status are device arrays of N entries.  The plan sorts
 * utterances longest first, picks each one's geometry from the tuning table,
 * uploads the descriptors, allocates the backpointer workspace and captures
 * the whole launch (queue reset + persistent kernel) in a HIP graph.
 * Alignments of up to 4096 states run as work items of the main persistent
 * kernel (a 4-wavefront workgroup runs one 4-wave alignment, or two 2-wave
 * or four 1-wave ones); larger ones (up to 32768 states) run
 * whole 8-wavefront workgroups of a second persistent kernel in the same
 * graph.
 * Emission rows must not straddle other utterances' outputs.
 * Errors: EINVAL (bad shape or pointer), ENOMEM, EDEVICE. */
int ctcalign_plan_create(ctcalign_ctx *ctx, int32_t N,
                         const float *emissions, const int64_t *em_off,
                         const int32_t *T, const int32_t *C,
                         const int32_t *labels, const int64_t *lab_off,
                         const int32_t *L, int32_t blank,
                         int32_t *out_paths, float *out_scores, const int64_t *frame_off,
                         float *out_totals, int32_t *out_status,
                         ctcalign_plan **plan);

/* Replays the plan's graph on `stream` (NULL: HIP's null stream).
 * Asynchronous; per-utterance statuses land in out_status.  A replay waits
 * for the plan's previous replay when that ran on another stream (they share
 * the plan's workspace). */
int ctcalign_plan_run(ctcalign_plan *plan, ctcalign_stream stream);

/* Profiling aid: when the plan was created with $CTCALIGN_TRACE=1, copies
 * (after its last run finished) the per-pack record {start, end, hardware id}
 * of the 100 MHz device wall clock into out_times[3*i..] and the instance
 * index run by each of the pack's 4 waves into out_insts[4*i..] (-1 idle),
 * for the first max_packs packs in queue order; *npacks gets the pack count.
 * EINVAL if the plan was created without tracing. */
int ctcalign_plan_trace(ctcalign_plan *plan, int32_t max_packs, int64_t *out_times,
                        int32_t *out_insts, int32_t *npacks);

/* Frees the plan (waits for its last run).  NULL is a no-op. */
int ctcalign_plan_destroy(ctcalign_plan *plan);

/* One-shot batched alignment: plan_create + plan_run + plan_destroy, with the
 * plan cached on the context while the same arguments come back. */
int ctcalign_align_batched(ctcalign_ctx *ctx, int32_t N,
                           const float *emissions, const int64_t *em_off,
                           const int32_t *T, const int32_t *C,
                           const int32_t *labels, const int64_t *lab_off,
                           const int32_t *L, int32_t blank,
                           int32_t *out_paths, float *out_scores, const int64_t *frame_off,
                           float *out_totals, int32_t *out_status,
                           ctcalign_stream stream);

/* ---- CTC prefix beam search with blank collapse ---------------------------
 * The paper's other GPU CTC kernel (Sec. 4, paragraph "CTC decoder"; Sec. 5,
 * "CUDA CTC decoder", Table 3): lexicon-free CTC prefix beam search without
 * a language model, every vocabulary class considered at every step, over
 * per-frame PROBABILITIES (softmax outputs, float32, in [0, 1]), after
 * blank collapse: a frame whose blank probability exceeds `threshold` is
 * dropped when the frame before it is such a frame too (so every run of
 * confident blank frames keeps its first frame; threshold >= 1 keeps every
 * frame).  Per kept frame, each hypothesis (a label prefix with p_b, p_nb)
 * stays (p_b' = (p_b + p_nb) * y[blank], p_nb' = p_nb * y[last]) or is
 * extended by each class c != blank (p_nb += (c == last ? p_b : p_b + p_nb)
 * * y[c], merged into an equal prefix already in the beam); the `beam`
 * candidates of largest total form the next beam (ties: stays and
 * extensions of better-ranked hypotheses first, then smaller classes).
 * Scores are kept relative to a running power of two, so long inputs never
 * underflow; every ranking decision and label is bitwise that of a plain
 * float32 evaluation in the same order (no fused multiply-add).
 *
 * N utterances; utterance i has T[i] frames of V classes at probs +
 * prob_off[i] (host arrays prob_off, T, tok_off).  Outputs (device):
 *   out_tokens + tok_off[i]   `beam` rows of T[i] labels: row k holds
 *                             hypothesis k's labels (out_len[i*beam + k] of them)
 *   out_len[i*beam + k]       label count (0 for k >= out_nhyp[i])
 *   out_logp[i*beam + k]      log-probability (nullable; -inf beyond out_nhyp)
 *   out_scaled / out_exp[i]   the total probability as scaled * 2^exp
 *                             (nullable; exact, for checking)
 *   out_nhyp[i]               hypotheses in the final beam (<= beam), in rank
 *                             order: row 0 is the decoded transcript
 *   out_nkept[i]              frames kept by blank collapse (nullable)
 *   out_status[i]             0, or 2 when no prefix keeps a positive
 *                             probability (out_nhyp = 0)
 * Limits: 2 <= V <= 1024, 1 <= beam <= 16.  One wavefront (a 64-thread
 * workgroup) per utterance, all utterances in one launch on `stream`.  workspace (device, 256-byte
 * aligned, >= ctcalign_beam_workspace_bytes) may be NULL: the context's
 * arena is used, ordered across streams as for ctcalign_align_ex.
 * Errors: EINVAL (arguments), ENOMEM, EDEVICE. */
int ctcalign_beam_decode(ctcalign_ctx *ctx, int32_t N, const float *probs, const int64_t *prob_off,
                         const int32_t *T, int32_t V, int32_t blank, int32_t beam, float threshold,
                         int32_t *out_tokens, const int64_t *tok_off, int32_t *out_len,
                         float *out_logp, float *out_scaled, int32_t *out_exp, int32_t *out_nhyp,
                         int32_t *out_nkept, int32_t *out_status, void *workspace, size_t ws_bytes,
                         ctcalign_stream stream);

/* Workspace bytes of ctcalign_beam_decode for N utterances of T[i] frames
 * (host array) and beam width `beam`; 0 on invalid arguments. */
size_t ctcalign_beam_workspace_bytes(int32_t N, const int32_t *T, int32_t beam);

/* ---- serving: continuous batching of arriving requests ------------------ */

/* One alignment request.  All pointers are device pointers that must stay
 * valid until the request's ticket completes; emission/labels as for
 * ctcalign_align_ex, out_total may be NULL.  ready_event (a hipEvent_t, or
 * NULL) is an event the caller recorded on the stream that writes the
 * emission and labels (and last used the outputs): the request is admitted
 * only once that event has completed, and requests behind it in the queue
 * wait with it (FIFO).  The event must stay valid until the ticket
 * completes.  With NULL the inputs must be written before the submit call. */
typedef struct ctcalign_request {
  const float *emission;
  int32_t T, C;
  const int32_t *labels;
  int32_t L, blank;
  int32_t *out_path;
  float *out_scores;
  float *out_total;
  void *ready_event;
} ctcalign_request;

/* Per-request timestamps, seconds on the host's monotonic clock
 * (CLOCK_MONOTONIC): submitted, admitted, launched, completion observed. */
typedef struct ctcalign_timing {
  double submit_s, admit_s, launch_s, done_s;
} ctcalign_timing;

typedef struct ctcalign_server_stats {
  uint64_t submitted, completed;
  uint64_t launches;         /* admitted groups handed to the resident kernel */
  uint64_t timeouts;         /* groups the watchdog gave up on */
  uint64_t readmitted;       /* requests queued again after a watchdog expiry */
  size_t peak_charge_bytes;  /* largest sum of charges in flight */
  size_t budget_bytes;
  int32_t peak_inflight, waiting, inflight;
  int32_t budget_violated;   /* 1 if the in-flight charge ever exceeded the budget */
} ctcalign_server_stats;

/* Starts a server on the context's device that runs alignments (paper
 * Sec. 4, "CTC-based forced alignment"; each request's result is bitwise
 * the one ctcalign_align_ex gives) as they arrive.  Each request is charged its
 * backpointer memory, T*(2L+1)/4 bytes (or its actual workspace if larger),
 * against bp_budget_bytes; requests are admitted in arrival order (FIFO)
 * while the charge in flight stays within the budget and fewer than
 * max_inflight requests are on the device.  Admitted requests run on a
 * resident kernel (one 16-wave workgroup per compute unit, or as many as
 * $CTCALIGN_SERVE_WGS says) that the server keeps on its own stream while
 * there is work and stops about 20 ms after the last request; each request
 * completes on its own, as soon as its alignment is written.  While that
 * kernel is resident it holds the compute units it runs on: other kernels
 * (and kernels the caller queues on a stream sharing its hardware queue)
 * wait for it to stop.
 * Requests hold up to S = 2L+1 = 16384 states.
 * Errors: EINVAL, ENOMEM (arena or pinned host memory), EDEVICE. */
int ctcalign_server_create(ctcalign_ctx *ctx, size_t bp_budget_bytes, int32_t max_inflight,
                           ctcalign_server **server);

/* Queues a request (never blocks).  *ticket identifies it.  Without a
 * ready_event the emission and labels must be written, and no other work may
 * write the outputs, before the call (the request may start at once).
 * Errors: EINVAL (bad arguments or 2L+1 > 16384; the request is not queued),
 * ENOMEM (its charge alone exceeds the budget), EAGAIN (queue full). */
int ctcalign_server_submit(ctcalign_server *server, const ctcalign_request *req, uint64_t *ticket);

/* Non-blocking completion check.  EBUSY while pending; OK once done, with
 * *status the alignment's own status (OK, EINVAL, EINFEASIBLE, or EDEVICE if
 * the watchdog gave up on it after 30 s or the kernel could not be launched)
 * and *timing filled (either may be NULL); the outputs are then written and
 * visible to any later work on the device.  A completed ticket is consumed by
 * the call; EINVAL for an unknown or consumed ticket. */
int ctcalign_server_poll(ctcalign_server *server, uint64_t ticket, int32_t *status,
                         ctcalign_timing *timing);

/* Like ctcalign_server_poll but waits for completion. */
int ctcalign_server_wait(ctcalign_server *server, uint64_t ticket, int32_t *status,
                         ctcalign_timing *timing);

/* Counters since creation. */
int ctcalign_server_get_stats(ctcalign_server *server, ctcalign_server_stats *stats);

/* Stops accepting requests, finishes every queued and running one, frees
 * the server.  NULL is a no-op. */
int ctcalign_server_destroy(ctcalign_server *server);

#ifdef __cplusplus
}
#endif
#endif /* CTCALIGN_H_ */
