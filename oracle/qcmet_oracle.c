/*
 * qcmet_oracle.c -- plain, slow, FP64 CPU reference of layered belief
 * propagation for QC-LDPC codes in syndrome form.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with
 * the GPU library.
 *
 * Paper: Li et al., "High-throughput GPU layered decoder of multi-edge type
 * LDPC codes in CV-QKD systems" (arXiv 2004.09084).
 *
 * What each routine follows:
 *   qo_phi            Methods, step 2: Phi(x) = -ln tanh(x/2), self-inverse.
 *   qo_clip           Results (kernel optimisations): messages are clipped to
 *                     keep Phi finite; the paper gives no constants, the
 *                     reading taken here is [Phi(30), 30].
 *   qo_greedy_schedule Results, merging of unrelated sub-matrices (the
 *                     examples Eq. (m), (m1), (m2)): rows that share no
 *                     block column form one layer.  Greedy rule: open a group
 *                     with the first unassigned row, add every later
 *                     unassigned row disjoint from the group, repeat.
 *   qo_decode_sp      Methods, steps 1-4 (layered sum-product, syndrome
 *                     form).  Per check: q = APP - r_old (step 3, first
 *                     equation, evaluated with the old r), the new r from
 *                     the other edges' q by the sign product and the Phi sum
 *                     (step 2), the syndrome flip (step 2, last equation),
 *                     APP = q + r_new (step 3), hard decision APP >= 0 -> 0
 *                     (step 4).  Every edge keeps its own message, degree-1
 *                     variables included: the oracle does not defer them.
 *                     msg_mode 1 rounds every new r to IEEE binary16
 *                     (round to nearest even) and keeps all else in FP64;
 *                     msg_mode 2 rounds it to an 8-bit float (4 exponent,
 *                     3 mantissa bits, round to nearest even).
 *   qo_decode_sp_early The same with early termination (Results, Table
 *                     tabearly): a frame stops at the first sweep count
 *                     whose hard decisions satisfy the syndrome.
 *   qo_decode_flood   Flooding schedule of the same sum-product update:
 *                     every check of an iteration reads the previous
 *                     iteration's APPs; then APP = LLR + sum of messages.
 *   qo_nms_*          Normalised/offset min-sum variant of the same layered
 *                     sweep (a learned decoder that is not in the paper):
 *                     r = sign * alpha[t][row][type] * max(min(min|q|, 30) - beta, 0);
 *                     the minimum saturates at the sum-product clip level
 *                     (Results, kernel optimisations: clipping keeps the
 *                     iterated values finite); analytic reverse-mode
 *                     gradients of the mean binary cross-entropy of the
 *                     final APP, or of its mean over the sweeps with each
 *                     term's gradient taken through a window of sweeps
 *                     (no gradient through an active clip).
 *
 * Parity pins (tests): brute-force bitwise MAP on cycle-free lifts, brute-
 * force ML on tiny loopy codes, single-check closed form (tanh rule),
 * degree-2 checks (r = +-q exactly), zero-noise and high-SNR frames, coset
 * symmetry, merged-vs-serial equality, numpy binary16 rounding, finite
 * differences of the NMS loss.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define QO_X_HI 30.0

/* Methods, step 2: Phi(x) = -ln(tanh(x/2)) = ln(1 + 2/(e^x - 1)). */
double qo_phi(double x) { return log1p(2.0 / expm1(x)); }

double qo_x_hi(void) { return QO_X_HI; }
double qo_x_lo(void) { return qo_phi(QO_X_HI); }

double qo_clip(double x) {
    double lo = qo_x_lo();
    if (x < lo) return lo;
    if (x > QO_X_HI) return QO_X_HI;
    return x;
}

/* IEEE-754 binary16, round to nearest, ties to even (1 sign bit, 5 exponent
 * bits, 10 fraction bits; subnormal quantum 2^-24; largest finite 65504). */
double qo_round_half(double v) {
    if (v == 0.0 || !isfinite(v)) return v;
    double a = fabs(v);
    int e;
    frexp(a, &e);               /* a in [2^(e-1), 2^e) */
    int qe = e - 11;            /* spacing of 11-bit significands in that binade */
    if (qe < -24) qe = -24;     /* subnormal range */
    double quantum = ldexp(1.0, qe);
    double r = nearbyint(a / quantum) * quantum;
    if (r > 65504.0) r = INFINITY;
    return copysign(r, v);
}

/* 8-bit float with 1 sign, 4 exponent (bias 7) and 3 mantissa bits, no
 * infinities, largest finite 448, subnormal spacing 2^-9 (the OCP e4m3
 * format): round to nearest, ties to even, from the definition; values
 * beyond 448 saturate. */
double qo_round_e4m3(double v) {
    if (v == 0.0 || !isfinite(v)) return v;
    double a = fabs(v);
    int e;
    frexp(a, &e);               /* a in [2^(e-1), 2^e) */
    int qe = e - 4;             /* spacing of 4-bit significands in that binade */
    if (qe < -9) qe = -9;       /* subnormal range (exponent -6, 3 fraction bits) */
    double quantum = ldexp(1.0, qe);
    double r = nearbyint(a / quantum) * quantum;
    if (r > 448.0) r = 448.0;
    return copysign(r, v);
}

/* ---------------------------------------------------------------- code -- */

typedef struct {
    int mb, nb, Z, n, m, E;
    const int *sh;        /* [mb*nb] */
    int *chk_ptr;         /* [m+1]  edges of check m: chk_ptr[m] .. chk_ptr[m+1]-1 */
    int *chk_vn;          /* [E]    variable node of each edge */
    int *chk_col;         /* [E]    base column of each edge */
    int *col_deg;         /* [nb]   non-(-1) entries per base column */
    int maxdeg;
} code_t;

static void code_free(code_t *c) {
    free(c->chk_ptr); free(c->chk_vn); free(c->chk_col); free(c->col_deg);
}

/* Edge (check i*Z+k) -- (variable j*Z + (k+a) mod Z) for each a = sh[i][j] >= 0,
 * edges of a check in ascending base column. */
static int code_build(code_t *c, int mb, int nb, int Z, const int *sh) {
    memset(c, 0, sizeof(*c));
    c->mb = mb; c->nb = nb; c->Z = Z; c->sh = sh;
    c->n = nb * Z; c->m = mb * Z;
    c->chk_ptr = (int *)malloc(sizeof(int) * (size_t)(c->m + 1));
    c->col_deg = (int *)calloc((size_t)nb, sizeof(int));
    if (!c->chk_ptr || !c->col_deg) return -1;
    int E = 0;
    for (int i = 0; i < mb; i++) {
        int rowdeg = 0;
        for (int j = 0; j < nb; j++) {
            int a = sh[i * nb + j];
            if (a >= Z || a < -1) return -2;
            if (a >= 0) { rowdeg++; c->col_deg[j]++; }
        }
        if (rowdeg > c->maxdeg) c->maxdeg = rowdeg;
        E += rowdeg * Z;
    }
    c->E = E;
    c->chk_vn = (int *)malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    c->chk_col = (int *)malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    if (!c->chk_vn || !c->chk_col) return -1;
    int e = 0;
    for (int i = 0; i < mb; i++) {
        for (int k = 0; k < Z; k++) {
            c->chk_ptr[i * Z + k] = e;
            for (int j = 0; j < nb; j++) {
                int a = sh[i * nb + j];
                if (a >= 0) {
                    c->chk_vn[e] = j * Z + (k + a) % Z;
                    c->chk_col[e] = j;
                    e++;
                }
            }
        }
    }
    c->chk_ptr[c->m] = e;
    return 0;
}

/* ------------------------------------------------------------ schedule -- */

static int rows_share_column(const int *sh, int nb, int r1, int r2) {
    for (int j = 0; j < nb; j++)
        if (sh[r1 * nb + j] >= 0 && sh[r2 * nb + j] >= 0) return 1;
    return 0;
}

/* Greedy merge of rows with disjoint block columns into layers.
 * Output: G, group_ptr[G+1], rows[mb] (rows of group g are
 * rows[group_ptr[g] .. group_ptr[g+1]-1], in ascending order). */
int qo_greedy_schedule(int mb, int nb, const int *sh, int *G, int *group_ptr, int *rows) {
    int *used = (int *)calloc((size_t)mb, sizeof(int));
    if (!used) return -1;
    int g = 0, p = 0;
    for (int first = 0; first < mb; first++) {
        if (used[first]) continue;
        group_ptr[g] = p;
        rows[p++] = first;
        used[first] = 1;
        for (int cand = first + 1; cand < mb; cand++) {
            if (used[cand]) continue;
            int clash = 0;
            for (int q = group_ptr[g]; q < p && !clash; q++)
                clash = rows_share_column(sh, nb, rows[q], cand);
            if (!clash) { rows[p++] = cand; used[cand] = 1; }
        }
        g++;
    }
    group_ptr[g] = p;
    *G = g;
    free(used);
    return 0;
}

/* Checks that (G, group_ptr, rows) lists every row exactly once and that the
 * rows of each group share no column.  0 if valid. */
int qo_check_schedule(int mb, int nb, const int *sh, int G, const int *group_ptr, const int *rows) {
    if (G < 0 || group_ptr[0] != 0 || group_ptr[G] != mb) return -1;
    int *seen = (int *)calloc((size_t)mb, sizeof(int));
    if (!seen) return -1;
    int bad = 0;
    for (int g = 0; g < G && !bad; g++) {
        if (group_ptr[g + 1] <= group_ptr[g]) bad = -1;
        for (int p = group_ptr[g]; p < group_ptr[g + 1] && !bad; p++) {
            int r = rows[p];
            if (r < 0 || r >= mb || seen[r]) { bad = -1; break; }
            seen[r] = 1;
            for (int q = group_ptr[g]; q < p; q++)
                if (rows_share_column(sh, nb, rows[q], r)) { bad = -2; break; }
        }
    }
    free(seen);
    return bad;
}

/* ---------------------------------------------------------- threading -- */

typedef struct {
    void (*fn)(void *ctx, int frame);
    void *ctx;
    int F, nth, tid;
} job_t;

static void *job_main(void *arg) {
    job_t *j = (job_t *)arg;
    for (int f = j->tid; f < j->F; f += j->nth) j->fn(j->ctx, f);
    return NULL;
}

/* Runs fn(ctx, f) for every frame f on nthreads threads (frames are
 * independent).  Returns the number of threads used. */
static int run_frames(void (*fn)(void *, int), void *ctx, int F, int nthreads) {
    if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > F) nthreads = F;
    if (nthreads <= 1) {
        for (int f = 0; f < F; f++) fn(ctx, f);
        return 1;
    }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    job_t *jobs = (job_t *)malloc(sizeof(job_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) {
        jobs[t].fn = fn; jobs[t].ctx = ctx; jobs[t].F = F; jobs[t].nth = nthreads; jobs[t].tid = t;
        pthread_create(&th[t], NULL, job_main, &jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th); free(jobs);
    return nthreads;
}

/* Step 4 and the syndrome test: c_n = [APP_n < 0]; flag = [H c == s]. */
static int hard_and_check(const code_t *c, const double *app, const uint8_t *s, uint8_t *hard) {
    for (int v = 0; v < c->n; v++) hard[v] = app[v] < 0.0 ? 1 : 0;
    for (int m = 0; m < c->m; m++) {
        int par = s[m] & 1;
        for (int e = c->chk_ptr[m]; e < c->chk_ptr[m + 1]; e++) par ^= hard[c->chk_vn[e]];
        if (par) return 0;
    }
    return 1;
}

/* ------------------------------------------------- layered sum-product -- */

typedef struct {
    const code_t *c;
    int G; const int *gptr, *rows;
    const float *llr; const uint8_t *syn;
    int T, mode, early_stop;
    double *app; uint8_t *hard, *flags;
    int32_t *iters;
    int err;
} sp_ctx;

static void sp_frame(void *vctx, int f) {
    sp_ctx *x = (sp_ctx *)vctx;
    const code_t *c = x->c;
    const int Z = c->Z, n = c->n, m = c->m;
    const float *llr = x->llr + (size_t)f * n;
    const uint8_t *s = x->syn + (size_t)f * m;
    double *app = x->app + (size_t)f * n;
    double *r = (double *)calloc((size_t)(c->E > 0 ? c->E : 1), sizeof(double));
    double *q = (double *)malloc(sizeof(double) * (size_t)(c->maxdeg + 1));
    double *ph = (double *)malloc(sizeof(double) * (size_t)(c->maxdeg + 1));
    double *rn = (double *)malloc(sizeof(double) * (size_t)(c->maxdeg + 1));
    if (!r || !q || !ph || !rn) { x->err = -1; free(r); free(q); free(ph); free(rn); return; }

    /* step 1: APP starts at the channel LLR 2R/sigma^2 (given); r = 0 */
    for (int v = 0; v < n; v++) app[v] = (double)llr[v];

    /* early termination (Results, Table tabearly): before every sweep the
     * hard decisions of the current APPs are tested against the syndrome and
     * the frame stops at the first sweep count where H c = s holds */
    uint8_t *hard = x->hard + (size_t)f * n;
    int used = 0;
    for (int t = 0; t < x->T; t++) {
        if (x->early_stop && hard_and_check(c, app, s, hard)) break;
        used = t + 1;
        for (int g = 0; g < x->G; g++) {
            for (int p = x->gptr[g]; p < x->gptr[g + 1]; p++) {
                int i = x->rows[p];
                for (int k = 0; k < Z; k++) {
                    int chk = i * Z + k;
                    int e0 = c->chk_ptr[chk], d = c->chk_ptr[chk + 1] - e0;
                    /* step 3, first equation: q_nm = APP_n - r_mn(old) */
                    for (int a = 0; a < d; a++) {
                        q[a] = app[c->chk_vn[e0 + a]] - r[e0 + a];
                        ph[a] = qo_phi(qo_clip(fabs(q[a])));
                    }
                    /* step 2: sign product and Phi sum over N(m) \ n, then
                     * the syndrome flip */
                    for (int a = 0; a < d; a++) {
                        double S = 0.0;
                        int neg = s[chk] & 1;
                        for (int b = 0; b < d; b++) {
                            if (b == a) continue;
                            S += ph[b];
                            neg ^= (q[b] < 0.0);
                        }
                        double mag = qo_phi(qo_clip(S));
                        double v = neg ? -mag : mag;
                        if (x->mode == 1) v = qo_round_half(v);
                        else if (x->mode == 2) v = qo_round_e4m3(v);
                        rn[a] = v;
                    }
                    /* step 3, second equation: APP_n = q_nm + r_mn(new) */
                    for (int a = 0; a < d; a++) {
                        r[e0 + a] = rn[a];
                        app[c->chk_vn[e0 + a]] = q[a] + rn[a];
                    }
                }
            }
        }
    }
    x->flags[f] = (uint8_t)hard_and_check(c, app, s, hard);
    if (x->iters) x->iters[f] = used;
    free(r); free(q); free(ph); free(rn);
}

/* Layered sum-product decode of F frames (frame-major buffers).
 *   llr  float [F][n]   channel LLRs (widened exactly to FP64)
 *   syn  uint8 [F][m]   syndrome bits
 *   T    iterations (full sweeps over all groups in schedule order)
 *   mode 0: FP64 messages; 1: messages rounded to binary16; 2: to e4m3
 *   app  double [F][n], hard uint8 [F][n], flags uint8 [F] (outputs)
 * Returns the number of threads used (>0) or a negative error. */
int qo_decode_sp(int mb, int nb, int Z, const int *sh, int G, const int *gptr, const int *rows,
                 int F, const float *llr, const uint8_t *syn, int T, int mode,
                 double *app, uint8_t *hard, uint8_t *flags, int nthreads) {
    if (mb <= 0 || nb <= 0 || Z <= 0 || F < 0 || T < 0 || mode < 0 || mode > 2) return -1;
    if (qo_check_schedule(mb, nb, sh, G, gptr, rows) != 0) return -3;
    code_t c;
    int rc = code_build(&c, mb, nb, Z, sh);
    if (rc) { code_free(&c); return rc; }
    sp_ctx x = {&c, G, gptr, rows, llr, syn, T, mode, 0, app, hard, flags, NULL, 0};
    int used = F > 0 ? run_frames(sp_frame, &x, F, nthreads) : 0;
    code_free(&c);
    return x.err ? x.err : (used > 0 ? used : 1);
}

/* The same decode with early termination: a frame stops after the first
 * sweep count t in [0, T] at which its hard decisions satisfy H c = s
 * (tested before every sweep and after the last); iters[f] = the sweeps it
 * ran.  A frame that stops at t has exactly the outputs of a T = t decode. */
int qo_decode_sp_early(int mb, int nb, int Z, const int *sh, int G, const int *gptr, const int *rows,
                       int F, const float *llr, const uint8_t *syn, int T, int mode,
                       double *app, uint8_t *hard, uint8_t *flags, int32_t *iters, int nthreads) {
    if (mb <= 0 || nb <= 0 || Z <= 0 || F < 0 || T < 0 || mode < 0 || mode > 2) return -1;
    if (qo_check_schedule(mb, nb, sh, G, gptr, rows) != 0) return -3;
    code_t c;
    int rc = code_build(&c, mb, nb, Z, sh);
    if (rc) { code_free(&c); return rc; }
    sp_ctx x = {&c, G, gptr, rows, llr, syn, T, mode, 1, app, hard, flags, iters, 0};
    int used = F > 0 ? run_frames(sp_frame, &x, F, nthreads) : 0;
    code_free(&c);
    return x.err ? x.err : (used > 0 ? used : 1);
}

/* ------------------------------------------------ flooding schedule -- */

/* Flooding sum-product (the schedule the paper sets layered decoding
 * against; Methods, steps 2-4 with every check of an iteration reading the
 * same APPs): per iteration, every check computes its new messages from
 * q = APP - r_old with the APPs of the previous iteration (step 2 rule,
 * syndrome flip, clip), then every variable takes APP = LLR + the sum of its
 * incoming messages, added in ascending check order.  The result does not
 * depend on the row order.  Outputs as qo_decode_sp. */
typedef struct {
    const code_t *c;
    const float *llr; const uint8_t *syn;
    int T, mode;
    double *app; uint8_t *hard, *flags;
    int err;
} flood_ctx;

static void flood_frame(void *vctx, int f) {
    flood_ctx *x = (flood_ctx *)vctx;
    const code_t *c = x->c;
    const int n = c->n, m = c->m;
    const float *llr = x->llr + (size_t)f * n;
    const uint8_t *s = x->syn + (size_t)f * m;
    double *app = x->app + (size_t)f * n;
    size_t E = (size_t)(c->E > 0 ? c->E : 1);
    double *r = (double *)calloc(E, sizeof(double));
    double *rn = (double *)malloc(sizeof(double) * E);
    double *q = (double *)malloc(sizeof(double) * (size_t)(c->maxdeg + 1));
    double *ph = (double *)malloc(sizeof(double) * (size_t)(c->maxdeg + 1));
    if (!r || !rn || !q || !ph) { x->err = -1; free(r); free(rn); free(q); free(ph); return; }
    for (int v = 0; v < n; v++) app[v] = (double)llr[v];
    for (int t = 0; t < x->T; t++) {
        /* every check from the same APPs */
        for (int chk = 0; chk < m; chk++) {
            int e0 = c->chk_ptr[chk], d = c->chk_ptr[chk + 1] - e0;
            for (int a = 0; a < d; a++) {
                q[a] = app[c->chk_vn[e0 + a]] - r[e0 + a];
                ph[a] = qo_phi(qo_clip(fabs(q[a])));
            }
            for (int a = 0; a < d; a++) {
                double S = 0.0;
                int neg = s[chk] & 1;
                for (int b = 0; b < d; b++) {
                    if (b == a) continue;
                    S += ph[b];
                    neg ^= (q[b] < 0.0);
                }
                double mag = qo_phi(qo_clip(S));
                double v = neg ? -mag : mag;
                if (x->mode == 1) v = qo_round_half(v);
                else if (x->mode == 2) v = qo_round_e4m3(v);
                rn[e0 + a] = v;
            }
        }
        /* every variable: LLR plus its messages, ascending check order */
        for (size_t e = 0; e < (size_t)c->E; e++) r[e] = rn[e];
        for (int v = 0; v < n; v++) app[v] = (double)llr[v];
        for (size_t e = 0; e < (size_t)c->E; e++) app[c->chk_vn[e]] += r[e];
    }
    x->flags[f] = (uint8_t)hard_and_check(c, app, s, x->hard + (size_t)f * n);
    free(r); free(rn); free(q); free(ph);
}

int qo_decode_flood(int mb, int nb, int Z, const int *sh, int F, const float *llr, const uint8_t *syn, int T,
                    int mode, double *app, uint8_t *hard, uint8_t *flags, int nthreads) {
    if (mb <= 0 || nb <= 0 || Z <= 0 || F < 0 || T < 0 || mode < 0 || mode > 2) return -1;
    code_t c;
    int rc = code_build(&c, mb, nb, Z, sh);
    if (rc) { code_free(&c); return rc; }
    flood_ctx x = {&c, llr, syn, T, mode, app, hard, flags, 0};
    int used = F > 0 ? run_frames(flood_frame, &x, F, nthreads) : 0;
    code_free(&c);
    return x.err ? x.err : (used > 0 ? used : 1);
}

/* ------------------------------------------------ normalised min-sum -- */

/* Weights: alpha, beta double [T][mb][2]; index 0 = target edge in a column
 * of degree >= 2 ("type-1"), 1 = target edge in a degree-1 column.  A check
 * with a single edge sees an empty minimum, read as X_HI; every minimum
 * saturates at X_HI. */

typedef struct {
    const code_t *c;
    int G; const int *gptr, *rows;
    const float *llr; const uint8_t *syn; const uint8_t *xbits;
    int T, early_stop;
    const double *alpha, *beta;
    double *app; uint8_t *hard, *flags; int32_t *iters;
    /* training */
    int want_grad;
    int every_sweep;       /* 0: loss on the APPs after the last sweep; 1: mean over sweeps */
    int window;            /* each loss term's gradient spans at most this many sweeps */
    double *loss_f;        /* [F] per-frame loss sums */
    double *ga_f, *gb_f;   /* [F][T*mb*2] per-frame gradient sums */
    int err;
} nms_ctx;

static int edge_type(const code_t *c, int e) { return c->col_deg[c->chk_col[e]] == 1 ? 1 : 0; }

static double dabs(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

/* softplus(u) = ln(1 + e^u) */
static double softplus(double u) { return (u > 0 ? u : 0.0) + log1p(exp(-fabs(u))); }
static double sigmoid(double u) { return u >= 0 ? 1.0 / (1.0 + exp(-u)) : exp(u) / (1.0 + exp(u)); }

/* exclusive minimum for edge a, saturated at X_HI: value and the lowest
 * index attaining it (-1 if the set is empty or the saturation is active) */
static double excl_min(const double *q, int d, int a, int *arg) {
    double mu = QO_X_HI;
    int best = -1;
    for (int b = 0; b < d; b++) {
        if (b == a) continue;
        double v = fabs(q[b]);
        if (best < 0 || v < mu) { mu = v; best = b; }
    }
    if (mu > QO_X_HI) {
        mu = QO_X_HI;
        best = -1;
    }
    *arg = best;
    return mu;
}

/* Loss term of one frame on its current APPs: adds softplus(-(1-2x) APP)
 * summed over the n bits, times wt, to *L, and sets gA to its derivative
 * with respect to each APP (the binary cross-entropy with
 * P(bit = 1) = sigmoid(-APP); the mean over frames and bits is taken by the
 * caller). */
static void nms_loss_term(const double *app, const uint8_t *xb, int n, double wt, double *L, double *gA) {
    double sum = 0.0;
    for (int v = 0; v < n; v++) {
        double sg = xb[v] ? -1.0 : 1.0;          /* 1 - 2x */
        sum += softplus(-sg * app[v]);
        gA[v] = -sg * sigmoid(-sg * app[v]);      /* d softplus(-sg A)/dA */
        gA[v] *= wt;
    }
    *L += wt * sum;
}

/* Reverse of sweep t of one frame, from its recorded q's (tape_t): gA holds
 * dL/dAPP after the sweep and gR dL/dr for the messages the sweep wrote (what
 * their later use as r_old sent back); on return they hold the same for the
 * state before the sweep.  Adds the weight gradients of sweep t into ga, gb. */
static void nms_backward_sweep(const nms_ctx *x, const uint8_t *s, const double *tape_t, int t, double *gA,
                               double *gR, double *ga, double *gb, double *q, double *gq, double *gr) {
    const code_t *c = x->c;
    const int Z = c->Z, mb = c->mb;
    for (int g = x->G - 1; g >= 0; g--) {
        for (int p = x->gptr[g + 1] - 1; p >= x->gptr[g]; p--) {
            int i = x->rows[p];
            for (int k = Z - 1; k >= 0; k--) {
                int chk = i * Z + k;
                int e0 = c->chk_ptr[chk], d = c->chk_ptr[chk + 1] - e0;
                for (int a = 0; a < d; a++) q[a] = tape_t[e0 + a];
                /* APP_new = q + r_new: both receive dL/dAPP_new; r_new
                 * also carries what its later use as r_old sent back */
                for (int a = 0; a < d; a++) {
                    int vn = c->chk_vn[e0 + a];
                    gq[a] = gA[vn];
                    gr[a] = gA[vn] + gR[e0 + a];
                }
                for (int a = 0; a < d; a++) {
                    int arg;
                    double mu = excl_min(q, d, a, &arg);
                    int neg = s[chk] & 1;
                    for (int b = 0; b < d; b++) if (b != a) neg ^= (q[b] < 0.0);
                    double sgn = neg ? -1.0 : 1.0;
                    int tau = edge_type(c, e0 + a);
                    size_t w = ((size_t)t * mb + (size_t)i) * 2 + (size_t)tau;
                    double z = mu - x->beta[w];
                    ga[w] += gr[a] * sgn * (z > 0.0 ? z : 0.0);
                    if (z > 0.0) {
                        double gz = gr[a] * sgn * x->alpha[w];
                        gb[w] -= gz;
                        if (arg >= 0) gq[arg] += gz * dabs(q[arg]);
                    }
                }
                /* q = APP_old - r_old */
                for (int a = 0; a < d; a++) {
                    gA[c->chk_vn[e0 + a]] = gq[a];
                    gR[e0 + a] = -gq[a];
                }
            }
        }
    }
}

static void nms_frame(void *vctx, int f) {
    nms_ctx *x = (nms_ctx *)vctx;
    const code_t *c = x->c;
    const int Z = c->Z, n = c->n, m = c->m, mb = c->mb, T = x->T;
    const float *llr = x->llr + (size_t)f * n;
    const uint8_t *s = x->syn + (size_t)f * m;
    double *app = x->app + (size_t)f * n;
    uint8_t *hard = x->hard + (size_t)f * n;
    size_t E = (size_t)(c->E > 0 ? c->E : 1);
    double *r = (double *)calloc(E, sizeof(double));
    double *tape = x->want_grad ? (double *)malloc(sizeof(double) * E * (size_t)(T > 0 ? T : 1)) : NULL;
    int D = c->maxdeg + 1;
    double *q = (double *)malloc(sizeof(double) * (size_t)D);
    double *rn = (double *)malloc(sizeof(double) * (size_t)D);
    double *gq = (double *)malloc(sizeof(double) * (size_t)D);
    double *gr = (double *)malloc(sizeof(double) * (size_t)D);
    double *gA = x->want_grad ? (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1)) : NULL;
    double *gR = x->want_grad ? (double *)malloc(sizeof(double) * E) : NULL;
    if (!r || !q || !rn || !gq || !gr || (x->want_grad && (!tape || !gA || !gR))) {
        x->err = -1; free(r); free(tape); free(q); free(rn); free(gq); free(gr); free(gA); free(gR); return;
    }
    const uint8_t *xb = x->want_grad ? x->xbits + (size_t)f * n : NULL;
    double *ga = x->want_grad ? x->ga_f + (size_t)f * (size_t)T * mb * 2 : NULL;
    double *gb = x->want_grad ? x->gb_f + (size_t)f * (size_t)T * mb * 2 : NULL;
    if (x->want_grad) x->loss_f[f] = 0.0;
    for (int v = 0; v < n; v++) app[v] = (double)llr[v];
    int used = 0;
    int ok = hard_and_check(c, app, s, hard);
    for (int t = 0; t < T; t++) {
        if (x->early_stop && ok) break;
        for (int g = 0; g < x->G; g++) {
            for (int p = x->gptr[g]; p < x->gptr[g + 1]; p++) {
                int i = x->rows[p];
                for (int k = 0; k < Z; k++) {
                    int chk = i * Z + k;
                    int e0 = c->chk_ptr[chk], d = c->chk_ptr[chk + 1] - e0;
                    for (int a = 0; a < d; a++) {
                        q[a] = app[c->chk_vn[e0 + a]] - r[e0 + a];
                        if (tape) tape[(size_t)t * E + (size_t)(e0 + a)] = q[a];
                    }
                    for (int a = 0; a < d; a++) {
                        int arg;
                        double mu = excl_min(q, d, a, &arg);
                        int neg = s[chk] & 1;
                        for (int b = 0; b < d; b++) if (b != a) neg ^= (q[b] < 0.0);
                        int tau = edge_type(c, e0 + a);
                        size_t w = ((size_t)t * mb + (size_t)i) * 2 + (size_t)tau;
                        double z = mu - x->beta[w];
                        double mag = x->alpha[w] * (z > 0.0 ? z : 0.0);
                        rn[a] = neg ? -mag : mag;
                    }
                    for (int a = 0; a < d; a++) {
                        r[e0 + a] = rn[a];
                        app[c->chk_vn[e0 + a]] = q[a] + rn[a];
                    }
                }
            }
        }
        used = t + 1;
        ok = hard_and_check(c, app, s, hard);
        if (x->want_grad && (x->every_sweep || t == T - 1)) {
            /* this sweep's loss term, then its gradient back through at most
             * `window` sweeps (t down to t - window + 1), holding the state
             * before the earliest of them fixed */
            nms_loss_term(app, xb, n, x->every_sweep ? 1.0 / (double)T : 1.0, &x->loss_f[f], gA);
            for (size_t e = 0; e < E; e++) gR[e] = 0.0;
            int lo = t - x->window + 1;
            if (lo < 0) lo = 0;
            for (int u = t; u >= lo; u--)
                nms_backward_sweep(x, s, tape + (size_t)u * E, u, gA, gR, ga, gb, q, gq, gr);
        }
    }
    ok = hard_and_check(c, app, s, hard);
    x->flags[f] = (uint8_t)ok;
    if (x->iters) x->iters[f] = used;

    free(r); free(tape); free(q); free(rn); free(gq); free(gr); free(gA); free(gR);
}

static int nms_run(int mb, int nb, int Z, const int *sh, int G, const int *gptr, const int *rows,
                   int F, const float *llr, const uint8_t *syn, const uint8_t *xbits, int T,
                   const double *alpha, const double *beta, int early_stop, int every_sweep, int window,
                   double *app, uint8_t *hard, uint8_t *flags, int32_t *iters,
                   double *loss, double *g_alpha, double *g_beta, int nthreads) {
    if (mb <= 0 || nb <= 0 || Z <= 0 || F < 0 || T < 0) return -1;
    if (window <= 0 || window > T) window = T;
    if (qo_check_schedule(mb, nb, sh, G, gptr, rows) != 0) return -3;
    code_t c;
    int rc = code_build(&c, mb, nb, Z, sh);
    if (rc) { code_free(&c); return rc; }
    int want = (loss != NULL);
    size_t W = (size_t)T * mb * 2;
    nms_ctx x;
    memset(&x, 0, sizeof(x));
    x.c = &c; x.G = G; x.gptr = gptr; x.rows = rows; x.llr = llr; x.syn = syn; x.xbits = xbits;
    x.T = T; x.early_stop = early_stop; x.alpha = alpha; x.beta = beta;
    x.app = app; x.hard = hard; x.flags = flags; x.iters = iters; x.want_grad = want;
    x.every_sweep = every_sweep; x.window = window;
    if (want) {
        x.loss_f = (double *)calloc((size_t)(F > 0 ? F : 1), sizeof(double));
        x.ga_f = (double *)calloc((size_t)(F > 0 ? F : 1) * (W > 0 ? W : 1), sizeof(double));
        x.gb_f = (double *)calloc((size_t)(F > 0 ? F : 1) * (W > 0 ? W : 1), sizeof(double));
        if (!x.loss_f || !x.ga_f || !x.gb_f) { code_free(&c); return -1; }
    }
    int used = F > 0 ? run_frames(nms_frame, &x, F, nthreads) : 1;
    if (want) {
        /* fixed-order sums over frames; mean over F*n bits */
        double norm = 1.0 / ((double)F * (double)c.n);
        double L = 0.0;
        for (int f = 0; f < F; f++) L += x.loss_f[f];
        *loss = L * norm;
        for (size_t w = 0; w < W; w++) {
            double a = 0.0, b = 0.0;
            for (int f = 0; f < F; f++) { a += x.ga_f[(size_t)f * W + w]; b += x.gb_f[(size_t)f * W + w]; }
            g_alpha[w] = a * norm;
            g_beta[w] = b * norm;
        }
        free(x.loss_f); free(x.ga_f); free(x.gb_f);
    }
    code_free(&c);
    return x.err ? x.err : used;
}

/* NMS decode, optionally stopping a frame once H c = s after a full
 * iteration (iters[f] = iterations run). */
int qo_nms_decode(int mb, int nb, int Z, const int *sh, int G, const int *gptr, const int *rows,
                  int F, const float *llr, const uint8_t *syn, int T,
                  const double *alpha, const double *beta, int early_stop,
                  double *app, uint8_t *hard, uint8_t *flags, int32_t *iters, int nthreads) {
    return nms_run(mb, nb, Z, sh, G, gptr, rows, F, llr, syn, NULL, T, alpha, beta, early_stop, 0, T,
                   app, hard, flags, iters, NULL, NULL, NULL, nthreads);
}

/* NMS forward over T fixed iterations, loss and analytic gradients.
 * every_sweep = 0: the loss is the mean BCE of the APPs after the last sweep;
 * 1: the mean over the T sweeps of the mean BCE of the APPs after each sweep.
 * window in [1, T] (anything else: T): the gradient of each loss term is
 * taken through at most that many sweeps, ending with the term's own, with
 * the state before the earliest of them held fixed; every_sweep = 0 with
 * window = T is the exact gradient of the final-sweep loss.
 * loss: scalar; g_alpha, g_beta: double [T][mb][2]. */
int qo_nms_train_grad(int mb, int nb, int Z, const int *sh, int G, const int *gptr, const int *rows,
                      int F, const float *llr, const uint8_t *syn, const uint8_t *xbits, int T,
                      const double *alpha, const double *beta, int every_sweep, int window,
                      double *app, double *loss, double *g_alpha, double *g_beta, int nthreads) {
    uint8_t *hard = (uint8_t *)malloc((size_t)(F > 0 ? F : 1) * (size_t)nb * (size_t)Z);
    uint8_t *flags = (uint8_t *)malloc((size_t)(F > 0 ? F : 1));
    if (!hard || !flags) { free(hard); free(flags); return -1; }
    int rc = nms_run(mb, nb, Z, sh, G, gptr, rows, F, llr, syn, xbits, T, alpha, beta, 0, every_sweep ? 1 : 0,
                     window, app, hard, flags, NULL, loss, g_alpha, g_beta, nthreads);
    free(hard); free(flags);
    return rc;
}

/* The exact gradient of the final-sweep loss (every_sweep = 0, window = T). */
int qo_nms_loss_grad(int mb, int nb, int Z, const int *sh, int G, const int *gptr, const int *rows,
                     int F, const float *llr, const uint8_t *syn, const uint8_t *xbits, int T,
                     const double *alpha, const double *beta,
                     double *app, double *loss, double *g_alpha, double *g_beta, int nthreads) {
    return qo_nms_train_grad(mb, nb, Z, sh, G, gptr, rows, F, llr, syn, xbits, T, alpha, beta, 0, T,
                             app, loss, g_alpha, g_beta, nthreads);
}
