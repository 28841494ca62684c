/*
 * CPU oracle for belief-propagation (BP) decoding of polar codes with
 * connected-sub-factor-graph (CSFG) freezing and G-matrix early stopping.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library.  It shares no code with the HIP path.
 *
 * Plain, slow and literal: every message column of the factor graph is kept,
 * loops run in the paper's order, and each function names the passage it
 * follows (Abbas, Fan, Chen, Tsui, "Low Complexity Belief Propagation Polar
 * Code Decoder").  The file is compiled twice: with REAL=float (the FP32
 * operation order the GPU must reproduce bit for bit) and with REAL=double
 * (the FP64 reference for error rates and gradients).  Build flags:
 * -O2 -ffp-contract=off, no fast-math (IEEE infinities carry meaning here).
 *
 * Notation (Section II-A): an (n,k) code with n = 2^m; the factor graph has
 * columns 1..m+1 (channel at column 1, source word u at column m+1) and rows
 * 0..n-1 (the paper counts rows from 1).  Stage j joins column j to column
 * j+1 and pairs rows (i, i + 2^{m-j}).  L[c][i] is the right-to-left message
 * and R[c][i] the left-to-right message of node (i, c).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

#ifndef REAL
#define REAL float
#endif
typedef REAL real;

typedef struct {
    int32_t max_iter;     /* maximum number of iterations (Section IV: 40) */
    int32_t early_stop;   /* 0: none (baseline BPD), 1: G-matrix check      */
    int32_t freezing;     /* 0: off, 1: CSFG freezing (Section III)         */
    int32_t freeze_input; /* 0: R alone (eq. 2 as printed), 1: R + L        */
    int32_t freeze_walk;  /* 0: one freeze per iteration, 1: one per stage,
                             2: greedy (keep checking after a freeze)       */
    double alpha;         /* min-sum scaling (Section IV: 0.9375)           */
    int32_t schedule;     /* 0: single left-to-right sweep (the reading of
                             Section II-A), 1: round trip (a right-to-left
                             pass of L, then a left-to-right pass of R)    */
} oracle_opts;

enum { WALK_ONE_PER_ITER = 0, WALK_ONE_PER_STAGE = 1, WALK_GREEDY = 2 };

int oracle_real_bytes(void) { return (int)sizeof(real); }

/* ------------------------------------------------------------------------
 * Encoding, Section II and Fig. 1: x = u F^{(x)m} with F = [[1,0],[1,1]],
 * computed by the XOR signal-flow graph: at every level h = 1, 2, ..., n/2
 * each node i whose bit h is clear takes x[i] ^ x[i+h].  The same network
 * computes eq. (3), since F^{(x)m} is its own inverse over GF(2).
 * ---------------------------------------------------------------------- */
void oracle_encode(int m, const uint8_t *u, uint8_t *x)
{
    int n = 1 << m;
    for (int i = 0; i < n; i++)
        x[i] = u[i] & 1;
    for (int h = 1; h < n; h <<= 1)
        for (int i = 0; i < n; i++)
            if (!(i & h))
                x[i] ^= x[i + h];
}

void oracle_encode_batch(int m, int64_t B, const uint8_t *u, uint8_t *x)
{
    int64_t n = (int64_t)1 << m;
    for (int64_t f = 0; f < B; f++)
        oracle_encode(m, u + f * n, x + f * n);
}

/* sign() of eq. (1): +1, -1, or 0 at zero. */
static real sgn(real v) { return (real)((v > 0) - (v < 0)); }

/* The scaled min-sum term of eq. (1): alpha * sign(x) * sign(y) *
 * min(|x|, |y|).  The sign factors are exact, so the product rounds once. */
static real gterm(real alpha, real x, real y)
{
    return alpha * sgn(x) * sgn(y) * fmin(fabs(x), fabs(y));
}

/* ------------------------------------------------------------------------
 * CSFG check, eqs. (2)-(4) and Lemma 1.  `in` holds the 2^{nlog} input
 * messages of one CSFG, `frozen` the frozen flags of its source-word rows.
 *   eq. (2): xhat = 1 where the message is < 0, else 0 (so -0 gives 0);
 *   eq. (3): uhat = xhat F^{(x)nlog};
 *   eq. (4): pass iff uhat is 0 at every frozen row.
 * Returns 1 on pass.  xhat/uhat receive the hard decisions.
 * ---------------------------------------------------------------------- */
int oracle_csfg_check(int nlog, const real *in, const uint8_t *frozen,
                      uint8_t *xhat, uint8_t *uhat)
{
    int n = 1 << nlog;
    for (int r = 0; r < n; r++)
        xhat[r] = in[r] < 0;
    oracle_encode(nlog, xhat, uhat);
    for (int r = 0; r < n; r++)
        if (uhat[r] && frozen[r])
            return 0;
    return 1;
}

/* Index of column c (1..m+1), row i. */
#define AT(c, i) ((size_t)(c) * (size_t)n + (size_t)(i))

/* ------------------------------------------------------------------------
 * Decode one frame.
 *
 * Schedule (Section II-A): per iteration t the PEs are activated stage by
 * stage from left to right; stage j computes L^t at column j from L^{t-1}
 * at column j+1 and R^t at column j, and R^t at column j+1, by eq. (1).
 * The round trip (schedule 1, no freezing) is the other common reading of
 * the same equations: per iteration, every L output of eq. (1) for stages
 * m, m-1, ..., 1, then every R output for stages 1, ..., m; each pass
 * counts as one activation of every PE.
 * Initial messages: R at column 1 = channel LLRs; L at column m+1 = +inf at
 * frozen rows and 0 at information rows; every other L = 0.
 *
 * Freezing (Section III): after stage j, the CSFGs at stage j (2^j of them,
 * the k-th taking R at column j+1 on rows [k 2^{m-j}, (k+1) 2^{m-j})) are
 * considered in decoded-bit order; a CSFG is checkable only when all CSFGs
 * before it at that stage are frozen, so the frozen CSFGs of a stage form a
 * prefix whose length is p[j].  A CSFG lying inside a frozen CSFG of an
 * earlier stage is frozen with it (p[j] >= 2 p[j-1]).  A check that fails
 * moves the walk to the next stage.  A CSFG that passes eqs. (2)-(4) is
 * frozen: its L at column j+1 becomes (-1)^xhat * inf for the rest of the
 * decoding, its decoded bits are kept, and the PEs inside it (stages > j on
 * its rows) are not activated again.  The walk policy after a successful
 * freeze is a reading (the paper leaves it open): one freeze per iteration,
 * one per stage, or greedy.
 *
 * Termination: all CSFGs of a stage frozen (then every source bit is
 * decided), the G-matrix check (uhat G equals the hard decision of the
 * total belief R + L at column 1), or max_iter.  Output bits are the hard
 * decision of R at column m+1 (frozen rows 0; rows inside frozen CSFGs take
 * the CSFG's decoded bits).
 *
 * PE count (Section IV): one per PE activation.
 * ---------------------------------------------------------------------- */
static int decode_frame(int m, const uint8_t *frozen, const float *llr,
                        const oracle_opts *o, uint8_t *uhat, int64_t *pe_out,
                        real *soft, int64_t frame, int32_t *trace,
                        int32_t trace_cap, int32_t *trace_len)
{
    const int n = 1 << m;
    const real alpha = (real)o->alpha;
    const real inf = (real)INFINITY;
    real *L = calloc((size_t)(m + 2) * n, sizeof(real));
    real *R = calloc((size_t)(m + 2) * n, sizeof(real));
    real *blk = malloc((size_t)n * sizeof(real));
    uint8_t *dec = calloc((size_t)n, 1);
    uint8_t *xh = malloc((size_t)n), *uh = malloc((size_t)n);
    uint8_t *xe = malloc((size_t)n);
    int *p = calloc((size_t)m + 1, sizeof(int));
    int64_t pe = 0;
    int t;

    for (int i = 0; i < n; i++) {
        R[AT(1, i)] = (real)llr[i];
        L[AT(m + 1, i)] = frozen[i] ? inf : (real)0;
    }

    for (t = 1; t <= o->max_iter; t++) {
        int walking = 1;
        if (o->schedule == 1) {
            /* round trip: eq. (1)'s L outputs for stages m..1 from the L
             * just computed at column j+1 and the R of the previous pass,
             * then its R outputs for stages 1..m from the R just computed
             * at column j and this pass's L at column j+1; every PE is
             * activated once in each pass */
            for (int j = m; j >= 1; j--) {
                const int h = n >> j;
                for (int a = 0; a < n; a++) {
                    if (a & h)
                        continue;
                    const int b = a + h;
                    const real La = L[AT(j + 1, a)], Lb = L[AT(j + 1, b)];
                    const real Ra = R[AT(j, a)], Rb = R[AT(j, b)];
                    L[AT(j, b)] = Lb + gterm(alpha, La, Ra);
                    L[AT(j, a)] = gterm(alpha, La, Lb + Rb);
                    pe++;
                }
            }
            for (int j = 1; j <= m; j++) {
                const int h = n >> j;
                for (int a = 0; a < n; a++) {
                    if (a & h)
                        continue;
                    const int b = a + h;
                    const real La = L[AT(j + 1, a)], Lb = L[AT(j + 1, b)];
                    const real Ra = R[AT(j, a)], Rb = R[AT(j, b)];
                    R[AT(j + 1, a)] = gterm(alpha, Ra, Lb + Rb);
                    R[AT(j + 1, b)] = Rb + gterm(alpha, La, Ra);
                    pe++;
                }
            }
        }
        for (int j = 1; j <= m && o->schedule == 0; j++) {
            const int h = n >> j;               /* 2^{m-j} */
            const int f = p[j - 1] * 2 * h;     /* frozen rows at column j */
            for (int a = f; a < n; a++) {
                if (a & h)
                    continue;
                const int b = a + h;
                const real La = L[AT(j + 1, a)], Lb = L[AT(j + 1, b)];
                const real Ra = R[AT(j, a)], Rb = R[AT(j, b)];
                /* eq. (1) */
                L[AT(j, b)] = Lb + gterm(alpha, La, Ra);
                L[AT(j, a)] = gterm(alpha, La, Lb + Rb);
                R[AT(j + 1, a)] = gterm(alpha, Ra, Lb + Rb);
                R[AT(j + 1, b)] = Rb + gterm(alpha, La, Ra);
                pe++;
            }
            if (!o->freezing)
                continue;
            if (p[j] < 2 * p[j - 1])
                p[j] = 2 * p[j - 1];
            while (p[j] < (1 << j)) {
                if (o->freeze_walk == WALK_ONE_PER_ITER && !walking)
                    break;
                const int k = p[j], r0 = k * h;
                int lg = m - j;
                for (int r = 0; r < h; r++)
                    blk[r] = o->freeze_input
                                 ? R[AT(j + 1, r0 + r)] + L[AT(j + 1, r0 + r)]
                                 : R[AT(j + 1, r0 + r)];
                int pass = oracle_csfg_check(lg, blk, frozen + r0, xh, uh);
                if (trace && *trace_len < trace_cap) {
                    int32_t *e = trace + 5 * (size_t)(*trace_len);
                    e[0] = (int32_t)frame; e[1] = t; e[2] = j; e[3] = k;
                    e[4] = pass;
                    (*trace_len)++;
                }
                if (!pass)
                    break;
                for (int r = 0; r < h; r++) {
                    L[AT(j + 1, r0 + r)] = xh[r] ? -inf : inf;
                    dec[r0 + r] = uh[r];
                }
                p[j] = k + 1;
                if (o->freeze_walk == WALK_ONE_PER_ITER) {
                    walking = 0;
                    break;
                }
                if (o->freeze_walk == WALK_ONE_PER_STAGE)
                    break;
            }
        }

        /* decisions at column m+1 */
        const int fm = o->freezing ? p[m] : 0;
        for (int i = 0; i < n; i++)
            uhat[i] = i < fm ? dec[i] : (frozen[i] ? 0 : R[AT(m + 1, i)] < 0);
        if (o->freezing && fm == n)
            break;
        if (o->early_stop) {
            /* G-matrix criterion: uhat G against the hard decision of the
             * total belief at the channel column */
            oracle_encode(m, uhat, xe);
            int same = 1;
            for (int i = 0; i < n && same; i++)
                same = xe[i] == (R[AT(1, i)] + L[AT(1, i)] < 0);
            if (same)
                break;
        }
    }
    if (t > o->max_iter)
        t = o->max_iter;

    if (soft) {
        const int fm = o->freezing ? p[m] : 0;
        for (int i = 0; i < n; i++)
            soft[i] = i < fm ? (dec[i] ? -inf : inf)
                             : R[AT(m + 1, i)] + L[AT(m + 1, i)];
    }
    *pe_out = pe;
    free(L); free(R); free(blk); free(dec); free(xh); free(uh); free(xe);
    free(p);
    return t;
}

/* Decode B frames of llr (B x n, row-major).  uhat: B x n source-word
 * decisions; iters: B; pe: B; soft (nullable): B x n posterior LLRs of u;
 * trace (nullable): 5 int32 per freezing check (frame, t, j, k, pass).
 * Returns 0, or -1 on bad arguments. */
int oracle_decode(int m, const uint8_t *frozen, int64_t B, const float *llr,
                  const oracle_opts *o, uint8_t *uhat, int32_t *iters,
                  int64_t *pe, real *soft, int32_t *trace, int32_t trace_cap,
                  int32_t *trace_len)
{
    if (m < 1 || m > 20 || B < 0 || !o || o->max_iter < 1 ||
        o->schedule < 0 || o->schedule > 1 || (o->schedule == 1 && o->freezing))
        return -1;
    int32_t dummy = 0;
    if (!trace_len)
        trace_len = &dummy;
    *trace_len = 0;
    const int64_t n = (int64_t)1 << m;
    for (int64_t f = 0; f < B; f++)
        iters[f] = decode_frame(m, frozen, llr + f * n, o, uhat + f * n,
                                pe + f, soft ? soft + f * n : NULL, f, trace,
                                trace_cap, trace_len);
    return 0;
}

/* ------------------------------------------------------------------------
 * Unrolled, trainable form: T iterations of the same single-sweep schedule
 * with no early stop and no freezing, where every (iteration t, stage j,
 * direction) owns its own scale in place of the single alpha of eq. (1):
 *   L^t_{a,j}   = aL * g0(L_a, L_b + R_b)      L^t_{b,j}   = L_b + aL * g0(L_a, R_a)
 *   R^t_{a,j+1} = aR * g0(R_a, L_b + R_b)      R^t_{b,j+1} = R_b + aR * g0(L_a, R_a)
 * with g0(x, y) = sign(x) sign(y) min(|x|, |y|), L = L^{t-1} at column j+1,
 * aL = alpha[(t-1) m 2 + (j-1) 2 + 0] and aR = alpha[... + 1].  With every
 * scale equal to 0.9375 this is plain T-iteration BP.  The output is R^T at
 * column m+1 (the posterior of the information rows).
 *
 * The gradient routine differentiates this forward map by reverse-mode
 * accumulation over the stored messages:
 *   d g0(x,y)/dx = sign(y) when |x| <= |y| (ties go to x), else 0;
 *   d g0(x,y)/dy = sign(x) when |x| >  |y|,                else 0;
 * and an infinite message is a constant (it neither receives a gradient nor
 * contributes to the scales' gradients).  Scales must be positive and finite
 * (a zero scale times an infinite message has no value).
 * ---------------------------------------------------------------------- */
static real g0(real x, real y) { return sgn(x) * sgn(y) * fmin(fabs(x), fabs(y)); }

/* Forward over one frame; keeps every column of every iteration in
 * Ls[t][c][i] (t = 0..T, L^0 = initial state) and Rs[t][c][i]. */
static void unrolled_fwd_frame(int m, const uint8_t *frozen, const float *llr,
                               int T, const double *alpha, real *Ls, real *Rs)
{
    const int n = 1 << m;
    const size_t col = (size_t)(m + 2) * n;
    const real inf = (real)INFINITY;
    memset(Ls, 0, sizeof(real) * col * (T + 1));
    memset(Rs, 0, sizeof(real) * col * (T + 1));
    for (int i = 0; i < n; i++)
        Ls[AT(m + 1, i)] = frozen[i] ? inf : (real)0;
    for (int t = 1; t <= T; t++) {
        real *Lp = Ls + col * (t - 1), *Lt = Ls + col * t, *Rt = Rs + col * t;
        for (int i = 0; i < n; i++) {
            Rt[AT(1, i)] = (real)llr[i];
            Lt[AT(m + 1, i)] = Lp[AT(m + 1, i)];
        }
        for (int j = 1; j <= m; j++) {
            const int h = n >> j;
            const real aL = (real)alpha[((size_t)(t - 1) * m + (j - 1)) * 2 + 0];
            const real aR = (real)alpha[((size_t)(t - 1) * m + (j - 1)) * 2 + 1];
            for (int a = 0; a < n; a++) {
                if (a & h)
                    continue;
                const int b = a + h;
                const real La = Lp[AT(j + 1, a)], Lb = Lp[AT(j + 1, b)];
                const real Ra = Rt[AT(j, a)], Rb = Rt[AT(j, b)];
                Lt[AT(j, a)] = aL * g0(La, Lb + Rb);
                Lt[AT(j, b)] = Lb + aL * g0(La, Ra);
                Rt[AT(j + 1, a)] = aR * g0(Ra, Lb + Rb);
                Rt[AT(j + 1, b)] = Rb + aR * g0(La, Ra);
            }
        }
    }
}

/* out: B x n, R^T at column m+1.  Returns 0, or -1 on bad arguments. */
int oracle_unrolled_forward(int m, const uint8_t *frozen, int64_t B,
                            const float *llr, int T, const double *alpha,
                            real *out)
{
    if (m < 1 || m > 16 || B < 0 || T < 1)
        return -1;
    const int n = 1 << m;
    const size_t col = (size_t)(m + 2) * n;
    real *Ls = malloc(sizeof(real) * col * (T + 1));
    real *Rs = malloc(sizeof(real) * col * (T + 1));
    for (int64_t f = 0; f < B; f++) {
        unrolled_fwd_frame(m, frozen, llr + f * n, T, alpha, Ls, Rs);
        const real *Rt = Rs + col * T;
        for (int i = 0; i < n; i++)
            out[f * n + i] = Rt[AT(m + 1, i)];
    }
    free(Ls); free(Rs);
    return 0;
}

/* Every message of the forward: L and R, each B x (T+1) x (m+2) x n, hold
 * column c of iteration t at [f][t][c][i] (t = 0 is the initial state;
 * column 0 is unused).  Returns 0, or -1 on bad arguments. */
int oracle_unrolled_messages(int m, const uint8_t *frozen, int64_t B,
                             const float *llr, int T, const double *alpha,
                             real *L, real *R)
{
    if (m < 1 || m > 16 || B < 0 || T < 1)
        return -1;
    const int n = 1 << m;
    const size_t per = (size_t)(m + 2) * n * (T + 1);
    for (int64_t f = 0; f < B; f++)
        unrolled_fwd_frame(m, frozen, llr + f * n, T, alpha, L + f * per,
                           R + f * per);
    return 0;
}

/* Route the adjoint d of g0(x, y) to x or y (see above); an infinite
 * operand takes nothing.  With mag set, the sign factor is dropped (see
 * unrolled_grad_core). */
static void g0_back(real x, real y, double d, double *dx, double *dy, int mag)
{
    if (fabs(x) <= fabs(y)) {
        if (isfinite(x))
            *dx += mag ? d : d * (double)sgn(y);
    } else {
        if (isfinite(y))
            *dy += mag ? d : d * (double)sgn(x);
    }
}

/* Gradients of sum_i dout[f][i] * out[f][i] with respect to the scales
 * (dalpha, T x m x 2, accumulated over frames) and to the channel LLRs
 * (dllr, B x n, nullable).  Both are written (not accumulated).
 *
 * Every gradient element is a sum, over the paths of the graph, of products
 * of a dout value, scales, signs and (for dalpha) one forward g0 value.
 * With mag set, the same accumulation runs on the magnitudes of those
 * factors (|dout|, no sign factors, |g0|): the result is the sum of the
 * magnitudes of the terms, the quantity that the rounding error of any
 * order of accumulating them is proportional to (a running-error bound for
 * sums of products).  It is not a gradient; it sizes the comparison of
 * gradients computed in another precision. */
static int unrolled_grad_core(int m, const uint8_t *frozen, int64_t B,
                              const float *llr, int T, const double *alpha,
                              const double *dout, double *dalpha,
                              double *dllr, int mag)
{
    if (m < 1 || m > 16 || B < 0 || T < 1)
        return -1;
    const int n = 1 << m;
    const size_t col = (size_t)(m + 2) * n;
    real *Ls = malloc(sizeof(real) * col * (T + 1));
    real *Rs = malloc(sizeof(real) * col * (T + 1));
    /* adjoints: dL[c][i] of L^t (current t), dR[c][i] of R^t */
    double *dL = malloc(sizeof(double) * col);
    double *dLprev = malloc(sizeof(double) * col);
    double *dR = malloc(sizeof(double) * col);
    memset(dalpha, 0, sizeof(double) * (size_t)T * m * 2);

    for (int64_t fr = 0; fr < B; fr++) {
        unrolled_fwd_frame(m, frozen, llr + fr * n, T, alpha, Ls, Rs);
        memset(dL, 0, sizeof(double) * col);
        double *dch = dllr ? dllr + fr * n : NULL;
        if (dch)
            memset(dch, 0, sizeof(double) * n);
        for (int t = T; t >= 1; t--) {
            const real *Lp = Ls + col * (t - 1), *Lt = Ls + col * t;
            const real *Rt = Rs + col * t;
            memset(dR, 0, sizeof(double) * col);
            memset(dLprev, 0, sizeof(double) * col);
            if (t == T)
                for (int i = 0; i < n; i++)
                    dR[AT(m + 1, i)] = mag ? fabs(dout[fr * n + i])
                                           : dout[fr * n + i];
            for (int j = m; j >= 1; j--) {
                const int h = n >> j;
                const size_t ai = ((size_t)(t - 1) * m + (j - 1)) * 2;
                const real aL = (real)alpha[ai], aR = (real)alpha[ai + 1];
                for (int a = 0; a < n; a++) {
                    if (a & h)
                        continue;
                    const int b = a + h;
                    const real La = Lp[AT(j + 1, a)], Lb = Lp[AT(j + 1, b)];
                    const real Ra = Rt[AT(j, a)], Rb = Rt[AT(j, b)];
                    const real s = Lb + Rb;
                    const real gA = g0(La, s), g1 = g0(La, Ra), gB = g0(Ra, s);
                    /* adjoints of the four outputs; infinite outputs are
                     * constants */
                    const int fLa = isfinite(Lt[AT(j, a)]);
                    const int fLb = isfinite(Lt[AT(j, b)]);
                    const int fRa = isfinite(Rt[AT(j + 1, a)]);
                    const int fRb = isfinite(Rt[AT(j + 1, b)]);
                    double oLa = fLa ? dL[AT(j, a)] : 0.0;
                    double oLb = fLb ? dL[AT(j, b)] : 0.0;
                    double oRa = fRa ? dR[AT(j + 1, a)] : 0.0;
                    double oRb = fRb ? dR[AT(j + 1, b)] : 0.0;
                    const double vA = mag ? fabs((double)gA) : (double)gA;
                    const double v1 = mag ? fabs((double)g1) : (double)g1;
                    const double vB = mag ? fabs((double)gB) : (double)gB;
                    if (fLa)
                        dalpha[ai + 0] += oLa * vA;
                    if (fLb)
                        dalpha[ai + 0] += oLb * v1;
                    if (fRa)
                        dalpha[ai + 1] += oRa * vB;
                    if (fRb)
                        dalpha[ai + 1] += oRb * v1;
                    double dgA = (double)aL * oLa;
                    double dg1 = (double)aL * oLb + (double)aR * oRb;
                    double dgB = (double)aR * oRa;
                    double dLa = 0, dLb = oLb, dRa = 0, dRb = oRb, ds = 0;
                    g0_back(La, s, dgA, &dLa, &ds, mag);
                    g0_back(La, Ra, dg1, &dLa, &dRa, mag);
                    g0_back(Ra, s, dgB, &dRa, &ds, mag);
                    if (isfinite(s)) {
                        dLb += ds;
                        dRb += ds;
                    }
                    if (isfinite(La))
                        dLprev[AT(j + 1, a)] += dLa;
                    if (isfinite(Lb))
                        dLprev[AT(j + 1, b)] += dLb;
                    dR[AT(j, a)] += dRa;
                    dR[AT(j, b)] += dRb;
                }
            }
            if (dch)
                for (int i = 0; i < n; i++)
                    dch[i] += dR[AT(1, i)];
            double *tmp = dL; dL = dLprev; dLprev = tmp;
        }
    }
    free(Ls); free(Rs); free(dL); free(dLprev); free(dR);
    return 0;
}

int oracle_unrolled_grad(int m, const uint8_t *frozen, int64_t B,
                         const float *llr, int T, const double *alpha,
                         const double *dout, double *dalpha, double *dllr)
{
    return unrolled_grad_core(m, frozen, B, llr, T, alpha, dout, dalpha, dllr,
                              0);
}

/* The magnitude sums of oracle_unrolled_grad's terms (mag mode above);
 * scales must be positive. */
int oracle_unrolled_grad_mag(int m, const uint8_t *frozen, int64_t B,
                             const float *llr, int T, const double *alpha,
                             const double *dout, double *dalpha, double *dllr)
{
    return unrolled_grad_core(m, frozen, B, llr, T, alpha, dout, dalpha, dllr,
                              1);
}

/* ------------------------------------------------------------------------
 * Successive-cancellation (SC) decoding: the decoder whose scheduling tree
 * Section III maps onto the factor graph (each CSFG of the BP graph is a
 * node of the SC tree, and Lemma 1's ML decision of a frozen CSFG is the
 * decision SC's subtree would reach no better than).  For G = F^{(x)m} in
 * natural order, G_n = F (x) G_{n/2}, so x = [(u_a ^ u_b) G_{n/2} |
 * u_b G_{n/2}] for the halves u_a, u_b of u.  A node of size n with the LLRs
 * L of its n codeword bits therefore decodes
 *   u_a from f(L[i], L[i + n/2])                     (the code u_a G_{n/2}),
 *   u_b from g(L[i], L[i + n/2], c_a[i]) = L[i + n/2] + (1 - 2 c_a[i]) L[i]
 *       with c_a = u_a G_{n/2}, the left subtree's re-encoded decisions,
 * and returns its own re-encoding [c_a ^ c_b | c_b].  f is the min-sum
 * check-node rule sign(a) sign(b) min(|a|, |b|) (exact: a selection, no
 * scaling); g rounds once.  A leaf takes u = 0 at a frozen position and
 * [LLR < 0] at an information position, in increasing index order.
 * ---------------------------------------------------------------------- */
static real sc_f(real a, real b) { return sgn(a) * sgn(b) * fmin(fabs(a), fabs(b)); }

static real sc_g(real a, real b, uint8_t c) { return b + (c ? -a : a); }

/* work: 2n reals; leaf: n reals (the LLR at each leaf) or NULL */
static void sc_node(int n, const real *L, const uint8_t *frozen, uint8_t *u,
                    uint8_t *x, real *work, real *leaf)
{
    if (n == 1) {
        if (leaf)
            leaf[0] = L[0];
        u[0] = frozen[0] ? 0 : (L[0] < 0);
        x[0] = u[0];
        return;
    }
    const int h = n / 2;
    real *Lc = work;            /* the child's n/2 LLRs */
    for (int i = 0; i < h; i++)
        Lc[i] = sc_f(L[i], L[i + h]);
    sc_node(h, Lc, frozen, u, x, work + h, leaf);
    for (int i = 0; i < h; i++)
        Lc[i] = sc_g(L[i], L[i + h], x[i]);
    sc_node(h, Lc, frozen + h, u + h, x + h, work + h, leaf ? leaf + h : NULL);
    for (int i = 0; i < h; i++)
        x[i] ^= x[i + h];
}

/* uhat: B x n source-word decisions; leaf: B x n leaf LLRs, or NULL.
 * Returns 0, or -1 on bad arguments. */
int oracle_sc_decode(int m, const uint8_t *frozen, int64_t B, const float *llr,
                     uint8_t *uhat, real *leaf)
{
    if (m < 0 || m > 20 || B < 0)
        return -1;
    const int n = 1 << m;
    real *L = malloc(sizeof(real) * (size_t)n);
    real *work = malloc(sizeof(real) * 2 * (size_t)n);
    uint8_t *x = malloc((size_t)n);
    for (int64_t f = 0; f < B; f++) {
        for (int i = 0; i < n; i++)
            L[i] = (real)llr[f * n + i];
        sc_node(n, L, frozen, uhat + f * n, x, work, leaf ? leaf + f * n : NULL);
    }
    free(L); free(work); free(x);
    return 0;
}

/* ------------------------------------------------------------------------
 * Fixed-point messages: the decoder of decode_frame (single sweep, early
 * stop, freezing) with every message a saturating b-bit integer, the form
 * in which the paper counts a PE's cost in hardware (Sections I and V).
 * The paper fixes no format; the reading:
 *   Q = 2^(b-1) - 1; every message lies in [-Q, Q];
 *   channel: q = clamp(round(LLR 2^F), -Q, Q), F fraction bits, rounding
 *            half away from zero;
 *   gq(x, y) = sign(x) sign(y) ((a min(|x|, |y|) + 8) >> 4),
 *            a = round(16 alpha) (15 for alpha = 0.9375): the scaled minimum
 *            rounded to the nearest integer, halves up (truncation would
 *            turn every magnitude-1 message into 0);
 *   sat(v) = clamp(v, -Q, Q) for every sum of eq. (1);
 *   +-inf of the frozen prior and of a frozen CSFG's L become +-Q;
 *   hard decisions (eq. (2), the stop test, the output) take the exact sum's
 *   sign: v < 0.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t bits;          /* message width b, 2..16 */
    int32_t frac;          /* fraction bits F of the channel quantizer */
} oracle_qfmt;

static int32_t q_sat(int32_t v, int32_t Q) { return v > Q ? Q : (v < -Q ? -Q : v); }

static int32_t q_sgn(int32_t v) { return (v > 0) - (v < 0); }

static int32_t q_g(int32_t a16, int32_t x, int32_t y)
{
    const int32_t ax = x < 0 ? -x : x, ay = y < 0 ? -y : y;
    const int32_t mn = ax < ay ? ax : ay;
    return q_sgn(x) * q_sgn(y) * ((a16 * mn + 8) >> 4);
}

/* one quantized channel value */
int32_t oracle_quantize(float llr, int32_t bits, int32_t frac)
{
    const int32_t Q = (1 << (bits - 1)) - 1;
    const double v = round((double)llr * ldexp(1.0, frac));
    return v > Q ? Q : (v < -Q ? -Q : (int32_t)v);
}

static int decode_frame_q(int m, const uint8_t *frozen, const float *llr,
                          const oracle_opts *o, const oracle_qfmt *qf,
                          uint8_t *uhat, int64_t *pe_out, int32_t *soft)
{
    const int n = 1 << m;
    const int32_t Q = (1 << (qf->bits - 1)) - 1;
    const int32_t a16 = (int32_t)lround(o->alpha * 16.0);
    int32_t *L = calloc((size_t)(m + 2) * n, sizeof(int32_t));
    int32_t *R = calloc((size_t)(m + 2) * n, sizeof(int32_t));
    uint8_t *dec = calloc((size_t)n, 1);
    uint8_t *xh = malloc((size_t)n), *uh = malloc((size_t)n);
    uint8_t *xe = malloc((size_t)n);
    int *p = calloc((size_t)m + 1, sizeof(int));
    int64_t pe = 0;
    int t;

    for (int i = 0; i < n; i++) {
        R[AT(1, i)] = oracle_quantize(llr[i], qf->bits, qf->frac);
        L[AT(m + 1, i)] = frozen[i] ? Q : 0;
    }
    for (t = 1; t <= o->max_iter; t++) {
        int walking = 1;
        for (int j = 1; j <= m; j++) {
            const int h = n >> j;
            const int f = p[j - 1] * 2 * h;
            for (int a = f; a < n; a++) {
                if (a & h)
                    continue;
                const int b = a + h;
                const int32_t La = L[AT(j + 1, a)], Lb = L[AT(j + 1, b)];
                const int32_t Ra = R[AT(j, a)], Rb = R[AT(j, b)];
                const int32_t s = q_sat(Lb + Rb, Q);
                L[AT(j, b)] = q_sat(Lb + q_g(a16, La, Ra), Q);
                L[AT(j, a)] = q_g(a16, La, s);
                R[AT(j + 1, a)] = q_g(a16, Ra, s);
                R[AT(j + 1, b)] = q_sat(Rb + q_g(a16, La, Ra), Q);
                pe++;
            }
            if (!o->freezing)
                continue;
            if (p[j] < 2 * p[j - 1])
                p[j] = 2 * p[j - 1];
            while (p[j] < (1 << j)) {
                if (o->freeze_walk == WALK_ONE_PER_ITER && !walking)
                    break;
                const int k = p[j], r0 = k * h;
                for (int r = 0; r < h; r++) {
                    const int32_t v = o->freeze_input
                                          ? R[AT(j + 1, r0 + r)] + L[AT(j + 1, r0 + r)]
                                          : R[AT(j + 1, r0 + r)];
                    xh[r] = v < 0;
                }
                oracle_encode(m - j, xh, uh);
                int pass = 1;
                for (int r = 0; r < h && pass; r++)
                    pass = !(uh[r] && frozen[r0 + r]);
                if (!pass)
                    break;
                for (int r = 0; r < h; r++) {
                    L[AT(j + 1, r0 + r)] = xh[r] ? -Q : Q;
                    dec[r0 + r] = uh[r];
                }
                p[j] = k + 1;
                if (o->freeze_walk == WALK_ONE_PER_ITER) {
                    walking = 0;
                    break;
                }
                if (o->freeze_walk == WALK_ONE_PER_STAGE)
                    break;
            }
        }
        const int fm = o->freezing ? p[m] : 0;
        for (int i = 0; i < n; i++)
            uhat[i] = i < fm ? dec[i] : (frozen[i] ? 0 : R[AT(m + 1, i)] < 0);
        if (o->freezing && fm == n)
            break;
        if (o->early_stop) {
            oracle_encode(m, uhat, xe);
            int same = 1;
            for (int i = 0; i < n && same; i++)
                same = xe[i] == (R[AT(1, i)] + L[AT(1, i)] < 0);
            if (same)
                break;
        }
    }
    if (t > o->max_iter)
        t = o->max_iter;
    if (soft) {
        const int fm = o->freezing ? p[m] : 0;
        for (int i = 0; i < n; i++)
            soft[i] = i < fm ? (dec[i] ? -Q : Q)
                             : q_sat(R[AT(m + 1, i)] + L[AT(m + 1, i)], Q);
    }
    *pe_out = pe;
    free(L); free(R); free(dec); free(xh); free(uh); free(xe); free(p);
    return t;
}

/* As oracle_decode (single sweep only) with fixed-point messages; soft
 * (nullable) receives sat(R + L) at column m+1 as integers. */
int oracle_decode_q(int m, const uint8_t *frozen, int64_t B, const float *llr,
                    const oracle_opts *o, const oracle_qfmt *qf, uint8_t *uhat,
                    int32_t *iters, int64_t *pe, int32_t *soft)
{
    if (m < 1 || m > 20 || B < 0 || !o || !qf || o->max_iter < 1 ||
        o->schedule != 0 || qf->bits < 2 || qf->bits > 16 || qf->frac < 0 ||
        qf->frac > 16)
        return -1;
    const int64_t n = (int64_t)1 << m;
    for (int64_t f = 0; f < B; f++)
        iters[f] = decode_frame_q(m, frozen, llr + f * n, o, qf, uhat + f * n,
                                  pe + f, soft ? soft + f * n : NULL);
    return 0;
}
