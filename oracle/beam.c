/*
 * CPU oracle for CTC prefix beam search with blank collapse -- TEST
 * INFRASTRUCTURE ONLY.  Only the test suite and the benchmark's CPU-baseline
 * leg may load this file's library; the product path never calls it.
 *
 * What it computes (paper Sec. 4, paragraph "CTC decoder": a CTC beam search
 * decoder, and a GPU version that parallelises over batch, hypotheses and
 * vocabulary and collapses blank frames; Sec. 5, "CUDA CTC decoder", Table 3:
 * beam 10, every vocabulary token considered at every step, blank frame skip
 * threshold a).  The paper prints no algorithm; this is the standard
 * lexicon-free CTC prefix beam search without a language model, written out
 * plainly: every hypothesis is a label prefix with two probabilities, p_b
 * (its frame paths end in a blank) and p_nb (they end in its last label).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *
 * 1. Inputs are per-frame probabilities y[t][c] (float32), not logs; all
 *    arithmetic is float32 multiply and add with round to nearest even, no
 *    fused multiply-add, denormals kept.  Probabilities are kept relative to
 *    a running power of two: after each frame every score is multiplied by
 *    2^-e, where the best candidate total is f * 2^e with f in [0.5, 1), and
 *    e is added to a running exponent E (multiplying by a power of two is
 *    exact while the result stays normal, and identical on any IEEE machine
 *    anyway).  The final log-probability of a hypothesis is
 *    log(p_b + p_nb) + E ln 2, evaluated in double.
 * 2. Blank collapse with threshold a: frame t is a blank frame when
 *    y[t][blank] > a (strictly, so a = 1 collapses nothing); in every maximal
 *    run of consecutive blank frames only the first frame is kept, the
 *    others are dropped before the search (one blank frame still separates
 *    repeated labels around the run).
 * 3. One step over a kept frame with probabilities y, for the beam
 *    h_0 .. h_{n-1} in rank order (s_j = p_b(h_j) + p_nb(h_j)):
 *      stay   h_j:      p_b'  = s_j * y[blank]
 *                       p_nb' = p_nb(h_j) * y[last(h_j)]  (0 for the empty prefix)
 *      extend h_i by c (c != blank):
 *                       x = (c == last(h_i) ? p_b(h_i) : s_i) * y[c]
 *        if h_i + c is already some beam hypothesis h_j, x joins h_j's stay:
 *                       p_nb'(h_j) = p_nb'(h_j) + x     (stay term first)
 *        else a new candidate with p_b' = 0, p_nb' = x.
 *    Candidate total = p_b' + p_nb'.  Candidates with total > 0 are ranked by
 *    total (descending), ties by key (ascending) where the key of h_j's stay
 *    is j * V + blank and that of "h_i extended by c" is i * V + c; the first
 *    B form the next beam.  Start: the empty prefix with p_b = 1, p_nb = 0.
 * 4. Output: the final beam in rank order, each hypothesis's labels and
 *    log-probability; the first is the decoded transcript.  If no candidate
 *    has a positive total the beam would be empty: status 2 (no hypothesis).
 *
 * Build: plain C, -O2, no fast-math, no FMA contraction.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BEAM_OK 0
#define BEAM_EINVAL 1
#define BEAM_ENOHYP 2
#define BEAM_ENOMEM 3

typedef struct {
    int32_t *tok;   /* labels of the prefix */
    int32_t len;
    float pb, pnb;
} Hyp;

typedef struct {
    int32_t src;    /* beam index of the hypothesis it comes from */
    int32_t c;      /* blank: stays with src; otherwise src extended by c */
    float pb, pnb, tot;
    int64_t key;
} Cand;

/* x * 2^k, exact while the result is normal; |k| steps of at most 126 keep
 * every factor representable. */
static float scale_pow2(float x, int k) {
    while (k > 126) { x = x * 0x1p126f; k -= 126; }
    while (k < -126) { x = x * 0x1p-126f; k += 126; }
    return x * ldexpf(1.0f, k);
}

/* Frames kept after blank collapse with threshold a; returns their count. */
int oracle_blank_collapse(const float *y, int32_t T, int32_t V, int32_t blank, float a,
                          int32_t *kept) {
    int32_t n = 0;
    int prev_blank = 0;
    for (int32_t t = 0; t < T; t++) {
        int is_blank = y[(int64_t)t * V + blank] > a;
        if (!(is_blank && prev_blank)) kept[n++] = t;
        prev_blank = is_blank;
    }
    return n;
}

static int cmp_cand(const void *pa, const void *pb) {
    const Cand *a = (const Cand *)pa, *b = (const Cand *)pb;
    if (a->tot > b->tot) return -1;
    if (a->tot < b->tot) return 1;
    return (a->key < b->key) ? -1 : (a->key > b->key);
}

/* h_j's prefix equals h_i's prefix followed by c */
static int is_extension(const Hyp *j, const Hyp *i, int32_t c) {
    if (j->len != i->len + 1 || j->tok[i->len] != c) return 0;
    return memcmp(j->tok, i->tok, sizeof(int32_t) * (size_t)i->len) == 0;
}

static void free_beam(Hyp *h, int n) {
    for (int k = 0; k < n; k++) free(h[k].tok);
}

/*
 * Decodes one utterance.  Outputs, for the final beam of *n_out <= B
 * hypotheses in rank order: out_len[k], labels at out_tok[k * T ..],
 * out_logp[k] (double), and (when not NULL) out_scaled[k] = p_b + p_nb as
 * kept (relative to 2^E) with *out_exp = E.  *n_kept receives the frame
 * count after blank collapse.
 */
int oracle_beam_decode_ex(const float *y, int32_t T, int32_t V, int32_t blank, int32_t B, float a,
                          int32_t *out_tok, int32_t *out_len, double *out_logp, float *out_scaled,
                          int32_t *out_exp, int32_t *n_out, int32_t *n_kept) {
    *n_out = 0;
    if (T < 1 || V < 2 || blank < 0 || blank >= V || B < 1) return BEAM_EINVAL;
    int32_t *kept = (int32_t *)malloc(sizeof(int32_t) * (size_t)T);
    Hyp *beam = (Hyp *)calloc((size_t)B, sizeof(Hyp));
    Hyp *next = (Hyp *)calloc((size_t)B, sizeof(Hyp));
    Cand *cand = (Cand *)malloc(sizeof(Cand) * (size_t)B * (size_t)V);
    if (!kept || !beam || !next || !cand) {
        free(kept); free(beam); free(next); free(cand);
        return BEAM_ENOMEM;
    }
    const int32_t nk = oracle_blank_collapse(y, T, V, blank, a, kept);
    *n_kept = nk;
    int n = 1;
    beam[0].tok = (int32_t *)malloc(sizeof(int32_t));
    beam[0].len = 0;
    beam[0].pb = 1.0f;
    beam[0].pnb = 0.0f;
    int64_t E = 0;
    int status = BEAM_OK;
    for (int32_t k = 0; k < nk && status == BEAM_OK; k++) {
        const float *yt = y + (int64_t)kept[k] * V;
        int nc = 0;
        /* stays first: candidate j is h_j's stay */
        for (int j = 0; j < n; j++) {
            const float s = beam[j].pb + beam[j].pnb;
            Cand *q = &cand[nc++];
            q->src = j;
            q->c = blank;
            q->pb = s * yt[blank];
            q->pnb = beam[j].len > 0 ? beam[j].pnb * yt[beam[j].tok[beam[j].len - 1]] : 0.0f;
            q->key = (int64_t)j * V + blank;
        }
        /* extensions, joining the stay of an existing hypothesis when equal */
        for (int i = 0; i < n; i++) {
            const float s = beam[i].pb + beam[i].pnb;
            const int32_t last = beam[i].len > 0 ? beam[i].tok[beam[i].len - 1] : -1;
            for (int32_t c = 0; c < V; c++) {
                if (c == blank) continue;
                const float x = (c == last ? beam[i].pb : s) * yt[c];
                int merged = -1;
                for (int j = 0; j < n; j++)
                    if (is_extension(&beam[j], &beam[i], c)) { merged = j; break; }
                if (merged >= 0) {
                    cand[merged].pnb = cand[merged].pnb + x;
                } else {
                    Cand *q = &cand[nc++];
                    q->src = i;
                    q->c = c;
                    q->pb = 0.0f;
                    q->pnb = x;
                    q->key = (int64_t)i * V + c;
                }
            }
        }
        int np = 0;
        for (int q = 0; q < nc; q++) {
            cand[q].tot = cand[q].pb + cand[q].pnb;
            if (cand[q].tot > 0.0f) cand[np++] = cand[q];
        }
        if (np == 0) { status = BEAM_ENOHYP; break; }
        qsort(cand, (size_t)np, sizeof(Cand), cmp_cand);
        const int m = np < B ? np : B;
        int e;
        (void)frexpf(cand[0].tot, &e);
        E += e;
        for (int r = 0; r < m; r++) {
            const Cand *q = &cand[r];
            const Hyp *h = &beam[q->src];
            const int ext = q->c != blank;
            next[r].len = h->len + ext;
            next[r].tok = (int32_t *)malloc(sizeof(int32_t) * (size_t)(next[r].len + 1));
            memcpy(next[r].tok, h->tok, sizeof(int32_t) * (size_t)h->len);
            if (ext) next[r].tok[h->len] = q->c;
            next[r].pb = scale_pow2(q->pb, -e);
            next[r].pnb = scale_pow2(q->pnb, -e);
        }
        free_beam(beam, n);
        Hyp *tmp = beam;
        beam = next;
        next = tmp;
        n = m;
    }
    if (status == BEAM_OK) {
        for (int r = 0; r < n; r++) {
            out_len[r] = beam[r].len;
            memcpy(out_tok + (int64_t)r * T, beam[r].tok, sizeof(int32_t) * (size_t)beam[r].len);
            const float tot = beam[r].pb + beam[r].pnb;
            out_logp[r] = log((double)tot) + (double)E * M_LN2;
            if (out_scaled) out_scaled[r] = tot;
        }
        if (out_exp) *out_exp = (int32_t)E;
        *n_out = n;
    }
    free_beam(beam, n);
    free(kept); free(beam); free(next); free(cand);
    return status;
}

int oracle_beam_decode(const float *y, int32_t T, int32_t V, int32_t blank, int32_t B, float a,
                       int32_t *out_tok, int32_t *out_len, double *out_logp, int32_t *n_out,
                       int32_t *n_kept) {
    return oracle_beam_decode_ex(y, T, V, blank, B, a, out_tok, out_len, out_logp, NULL, NULL,
                                 n_out, n_kept);
}

/* ---- many utterances on POSIX threads -------------------------------------- */

typedef struct {
    int32_t n, V, blank, B;
    float a;
    const float *y;
    const int64_t *y_off, *tok_off;
    const int32_t *T;
    int32_t *out_tok, *out_len, *n_out, *n_kept, *status, *out_exp;
    double *out_logp;
    float *out_scaled;
    int next;
    pthread_mutex_t mu;
} BatchJob;

static void *batch_worker(void *arg) {
    BatchJob *J = (BatchJob *)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        const int i = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (i >= J->n) break;
        J->status[i] = oracle_beam_decode_ex(J->y + J->y_off[i], J->T[i], J->V, J->blank, J->B,
                                             J->a, J->out_tok + J->tok_off[i],
                                             J->out_len + (int64_t)i * J->B,
                                             J->out_logp + (int64_t)i * J->B,
                                             J->out_scaled + (int64_t)i * J->B, J->out_exp + i,
                                             J->n_out + i, J->n_kept + i);
    }
    return NULL;
}

/* Utterance i: probabilities at y + y_off[i] ([T[i]][V]); its final beam goes
 * to out_tok + tok_off[i] (B rows of T[i] labels), out_len / out_logp /
 * out_scaled [i*B ..], out_exp[i], n_out[i], n_kept[i], status[i].  Returns
 * the threads used. */
int oracle_beam_decode_batch(int32_t n, const float *y, const int64_t *y_off, const int32_t *T,
                             int32_t V, int32_t blank, int32_t B, float a, int32_t *out_tok,
                             const int64_t *tok_off, int32_t *out_len, double *out_logp,
                             float *out_scaled, int32_t *out_exp, int32_t *n_out, int32_t *n_kept,
                             int32_t *status, int32_t threads) {
    BatchJob J = {n, V, blank, B, a, y, y_off, tok_off, T, out_tok, out_len, n_out, n_kept,
                  status, out_exp, out_logp, out_scaled, 0, PTHREAD_MUTEX_INITIALIZER};
    if (threads < 1) threads = 1;
    if (threads > n) threads = n > 0 ? n : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    int used = 0;
    for (int k = 0; k < threads; k++)
        if (pthread_create(&th[k], NULL, batch_worker, &J) == 0) used++;
    if (used == 0) batch_worker(&J);
    for (int k = 0; k < used; k++) pthread_join(th[k], NULL);
    free(th);
    return used > 0 ? used : 1;
}
