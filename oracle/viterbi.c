/*
 * CPU oracle for CTC forced alignment -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this file's library.  The product path never calls it.
 *
 * What it computes (paper Sec. 4, paragraph "CTC-based forced alignment":
 * frame-level alignment of a transcript to the per-frame outputs of a
 * CTC-trained network; the CTC formalism is Graves et al. 2006, cited in the
 * paper's introduction).  Forced alignment is the Viterbi maximum over all
 * CTC paths that collapse to the transcript, computed here on the
 * blank-interleaved trellis exactly as its definition reads, one state at a
 * time, with no blocking or reordering:
 *
 *   S = 2L+1;  y'_s = blank for even s,  y'_s = y_{(s-1)/2} for odd s
 *   skip(s)  = s odd, s >= 3, y'_s != y'_{s-2}
 *   a_0(s)   = E[0, y'_s] for s in {0, 1}, -inf otherwise
 *   for t = 1..T-1, s = 0..S-1:
 *       best = a_{t-1}(s), k = 0
 *       if s >= 1 and a_{t-1}(s-1) > best:      best = a_{t-1}(s-1), k = 1
 *       if skip(s) and a_{t-1}(s-2) > best:     best = a_{t-1}(s-2), k = 2
 *       a_t(s) = E[t, y'_s] + best   (one IEEE add, round to nearest even)
 *       bp_t(s) = k
 *   end state: S == 1 -> 0; else S-2 if a_{T-1}(S-2) > a_{T-1}(S-1), else S-1
 *   total = a_{T-1}(end);  -inf -> infeasible
 *   backtrack s_{t-1} = s_t - bp_t(s_t);  path[t] = y'_{s_t};
 *   scores[t] = E[t, path[t]]
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes): initialisation as above; ties keep the lower displacement (strict
 * '>' in the order s, s-1, s-2); the end-state tie keeps S-1; L = 0 is
 * allowed (all-blank path); an infeasible input returns status 2 with
 * path = -1, scores = -inf, total = -inf; a label equal to the blank or out
 * of [0, C) returns status 1 with path = -1, scores = NaN.
 *
 * Two precisions: the float variant keeps a_t in float and performs exactly
 * one float add per state and frame (the reference arithmetic for bitwise
 * parity); the double variant upcasts E exactly and runs the same steps in
 * double (for the cross-precision tolerance check only).
 *
 * Build: plain C, -O2, no fast-math, no FMA contraction, no flush-to-zero.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_EINFEASIBLE 2
#define ORACLE_ENOMEM 3

static int yprime(const int32_t *y, int32_t blank, int64_t s) {
    return (s % 2 == 0) ? blank : y[(s - 1) / 2];
}

/* Labels must be class ids in [0, C) other than the blank. */
static int check_labels(const int32_t *y, int32_t L, int32_t C, int32_t blank) {
    for (int32_t i = 0; i < L; i++)
        if (y[i] < 0 || y[i] >= C || y[i] == blank) return ORACLE_EINVAL;
    return ORACLE_OK;
}

/* Float variant.  `total` may be NULL. */
int oracle_align_f32(const float *E, int32_t T, int32_t C, const int32_t *y,
                     int32_t L, int32_t blank, int32_t *path, float *scores,
                     float *total) {
    if (!E || !path || !scores || T < 1 || C < 1 || L < 0 || blank < 0 ||
        blank >= C || (L > 0 && !y))
        return ORACLE_EINVAL;
    if (check_labels(y, L, C, blank) != ORACLE_OK) {
        for (int32_t t = 0; t < T; t++) { path[t] = -1; scores[t] = NAN; }
        if (total) *total = NAN;
        return ORACLE_EINVAL;
    }
    const int64_t S = 2 * (int64_t)L + 1;
    float *prev = (float *)malloc(sizeof(float) * S);
    float *cur = (float *)malloc(sizeof(float) * S);
    uint8_t *bp = (uint8_t *)malloc((size_t)T * (size_t)S);
    if (!prev || !cur || !bp) { free(prev); free(cur); free(bp); return ORACLE_ENOMEM; }

    for (int64_t s = 0; s < S; s++)
        prev[s] = (s <= 1) ? E[yprime(y, blank, s)] : -INFINITY;

    for (int32_t t = 1; t < T; t++) {
        const float *Et = E + (int64_t)t * C;
        uint8_t *bpt = bp + (int64_t)t * S;
        for (int64_t s = 0; s < S; s++) {
            float best = prev[s];
            uint8_t k = 0;
            if (s >= 1 && prev[s - 1] > best) { best = prev[s - 1]; k = 1; }
            if (s % 2 == 1 && s >= 3 && yprime(y, blank, s) != yprime(y, blank, s - 2) &&
                prev[s - 2] > best) { best = prev[s - 2]; k = 2; }
            cur[s] = Et[yprime(y, blank, s)] + best;   /* one float add */
            bpt[s] = k;
        }
        float *tmp = prev; prev = cur; cur = tmp;
    }

    int64_t send = 0;
    if (S > 1) send = (prev[S - 2] > prev[S - 1]) ? S - 2 : S - 1;
    const float tot = prev[send];
    int status = ORACLE_OK;
    if (tot == -INFINITY) {
        status = ORACLE_EINFEASIBLE;
        for (int32_t t = 0; t < T; t++) { path[t] = -1; scores[t] = -INFINITY; }
    } else {
        int64_t s = send;
        for (int32_t t = T - 1; t >= 0; t--) {
            int c = yprime(y, blank, s);
            path[t] = c;
            scores[t] = E[(int64_t)t * C + c];
            if (t > 0) s -= bp[(int64_t)t * S + s];
        }
    }
    if (total) *total = tot;
    free(prev); free(cur); free(bp);
    return status;
}

/* Double variant: same steps, E upcast exactly to double, a_t in double. */
int oracle_align_f64(const float *E, int32_t T, int32_t C, const int32_t *y,
                     int32_t L, int32_t blank, int32_t *path, double *scores,
                     double *total) {
    if (!E || !path || !scores || T < 1 || C < 1 || L < 0 || blank < 0 ||
        blank >= C || (L > 0 && !y))
        return ORACLE_EINVAL;
    if (check_labels(y, L, C, blank) != ORACLE_OK) {
        for (int32_t t = 0; t < T; t++) { path[t] = -1; scores[t] = NAN; }
        if (total) *total = NAN;
        return ORACLE_EINVAL;
    }
    const int64_t S = 2 * (int64_t)L + 1;
    double *prev = (double *)malloc(sizeof(double) * S);
    double *cur = (double *)malloc(sizeof(double) * S);
    uint8_t *bp = (uint8_t *)malloc((size_t)T * (size_t)S);
    if (!prev || !cur || !bp) { free(prev); free(cur); free(bp); return ORACLE_ENOMEM; }

    for (int64_t s = 0; s < S; s++)
        prev[s] = (s <= 1) ? (double)E[yprime(y, blank, s)] : -INFINITY;

    for (int32_t t = 1; t < T; t++) {
        const float *Et = E + (int64_t)t * C;
        uint8_t *bpt = bp + (int64_t)t * S;
        for (int64_t s = 0; s < S; s++) {
            double best = prev[s];
            uint8_t k = 0;
            if (s >= 1 && prev[s - 1] > best) { best = prev[s - 1]; k = 1; }
            if (s % 2 == 1 && s >= 3 && yprime(y, blank, s) != yprime(y, blank, s - 2) &&
                prev[s - 2] > best) { best = prev[s - 2]; k = 2; }
            cur[s] = (double)Et[yprime(y, blank, s)] + best;
            bpt[s] = k;
        }
        double *tmp = prev; prev = cur; cur = tmp;
    }

    int64_t send = 0;
    if (S > 1) send = (prev[S - 2] > prev[S - 1]) ? S - 2 : S - 1;
    const double tot = prev[send];
    int status = ORACLE_OK;
    if (tot == -INFINITY) {
        status = ORACLE_EINFEASIBLE;
        for (int32_t t = 0; t < T; t++) { path[t] = -1; scores[t] = -INFINITY; }
    } else {
        int64_t s = send;
        for (int32_t t = T - 1; t >= 0; t--) {
            int c = yprime(y, blank, s);
            path[t] = c;
            scores[t] = (double)E[(int64_t)t * C + c];
            if (t > 0) s -= bp[(int64_t)t * S + s];
        }
    }
    if (total) *total = tot;
    free(prev); free(cur); free(bp);
    return status;
}

/* ---- many utterances over a pool of POSIX threads (for timing only) ------ */

typedef struct {
    int32_t n;
    const float *em; const int64_t *em_off;
    const int32_t *T; const int32_t *C;
    const int32_t *lab; const int64_t *lab_off; const int32_t *L;
    int32_t blank;
    int32_t *paths; float *scores; const int64_t *fr_off;
    float *totals; int32_t *status;
    int32_t next;               /* shared work counter */
    pthread_mutex_t mu;
} batch_job;

static void *batch_worker(void *arg) {
    batch_job *j = (batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int32_t i = j->next++;
        pthread_mutex_unlock(&j->mu);
        if (i >= j->n) break;
        j->status[i] = oracle_align_f32(j->em + j->em_off[i], j->T[i], j->C[i],
                                        j->lab + j->lab_off[i], j->L[i], j->blank,
                                        j->paths + j->fr_off[i], j->scores + j->fr_off[i],
                                        j->totals + i);
    }
    return NULL;
}

/* Aligns n utterances (float variant) on `threads` threads, one utterance per
 * task, taken in index order.  Returns the number of threads used. */
int oracle_align_batch_f32(int32_t n, const float *em, const int64_t *em_off,
                           const int32_t *T, const int32_t *C, const int32_t *lab,
                           const int64_t *lab_off, const int32_t *L, int32_t blank,
                           int32_t *paths, float *scores, const int64_t *fr_off,
                           float *totals, int32_t *status, int32_t threads) {
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    batch_job j = {n, em, em_off, T, C, lab, lab_off, L, blank, paths, scores,
                   fr_off, totals, status, 0, PTHREAD_MUTEX_INITIALIZER};
    pthread_t tid[256];
    int started = 0;
    for (int k = 1; k < threads; k++)
        if (pthread_create(&tid[started], NULL, batch_worker, &j) == 0) started++;
    batch_worker(&j);
    for (int k = 0; k < started; k++) pthread_join(tid[k], NULL);
    return started + 1;
}
