/*
 * arsel CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, obviously-correct CPU implementation of what the
 * selection path computes.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path never
 * does.  It shares no code, header or table with the HIP sources.
 *
 * What it follows (Neri & Mestivier, "An efficient GPU acceptance-rejection
 * algorithm for the selection of the next reaction to occur for Stochastic
 * Simulation Algorithms", arXiv:1404.0027):
 *
 *  - Section "A GPU acceptance-rejection algorithm (GPU/AR) for SSA", first
 *    paragraph: the sequential acceptance-rejection rule -- draw a reaction
 *    index j uniformly and a uniform u in [0,T) until u < alpha_j; the first
 *    accepted candidate is the next reaction.  Here T = alpha_max (or a
 *    caller-supplied bound >= alpha_max), and the draw sequence is indexed by
 *    an explicit trial counter t = 0, 1, ... so the answer is "the accepted
 *    candidate with the least t".  Trials are capped at t_max.
 *  - Section "The Stochastic Simulation Algorithm": the inverse-transform
 *    rule (least j whose cumulative propensity exceeds r * alpha_0), used
 *    here, in exact fixed-point integers, as the fallback when t_max trials
 *    all reject.
 *  - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 *    random numbers: as easy as 1, 2, 3", SC'11), written here from that
 *    published definition.  The paper itself only names the GPU generators
 *    it used (section "Materials").
 *  - Section "The Stochastic Simulation Algorithm" again for the SSA state
 *    update X <- X + v_j used by the jump-chain data generator, and for the
 *    direct method's time step tau = ln(1/u) / alpha_0 of the full SSA run,
 *    with ln by Tang's published table-driven method and alpha_0 summed
 *    exactly in 128-bit fixed point, then rounded once (both fixed below).
 *
 * Readings where the paper is silent are listed in the design notes; the
 * ones that fix arithmetic here: one Philox block b yields two trials,
 * t = 2b (words 0, 1) and t = 2b+1 (words 2, 3); in each trial the first
 * word picks the candidate and the second is u on the 32-bit grid
 * {0, 2^-32, ..., 1 - 2^-32}; the product u*alpha_max is one binary64
 * multiply (a 24-bit float grid would over-weight reactions with
 * alpha_j < 2^-24 alpha_max); acceptance is strict (u*alpha_max < alpha_j);
 * candidates are
 * exactly uniform (Lemire multiply-shift with its rejection folded into the
 * trial); indexes are 0-based; -1 means every propensity is zero and -2 an
 * invalid (NaN, negative, +inf) propensity.
 *
 * Build: gcc -O2 -std=gnu11 -ffp-contract=off -fopenmp -shared -fPIC.  No
 * fast-math, default MXCSR (no FTZ/DAZ), so every float op is one IEEE op.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): counter c[4], key k[2]; 10 rounds; after each */
/* round the key is bumped by the two Weyl constants.                   */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout of one random draw: (word0, instance, step lo, step hi ^ tag<<28).
 * Tags: 0 uniform select, 1 proposal select, 2 SSA data generation.
 * word0 is the trial block t/2; 0xFFFFFFFF is reserved for the fallback draw. */
#define FALLBACK_WORD 0xFFFFFFFFu

static void draw(uint64_t seed, uint32_t word0, uint32_t inst, uint64_t step,
                 uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = { word0, inst, (uint32_t)step,
                        (uint32_t)(step >> 32) ^ (tag << 28) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    orc_philox4x32_10(ctr, key, out);
}

/* u on the 32-bit grid {0, 2^-32, ..., 1 - 2^-32}, exact in binary64. */
static double grid_u(uint32_t w)
{
    return (double)w * 0x1p-32;
}

/* Trial t: candidate word and u word. */
static void trial_words(uint64_t seed, uint32_t t, uint32_t inst, uint64_t step,
                        uint32_t tag, uint32_t *cand, uint32_t *uw)
{
    uint32_t w[4];
    draw(seed, t >> 1, inst, step, tag, w);
    *cand = w[2 * (t & 1)];
    *uw = w[2 * (t & 1) + 1];
}

/* L = ceil(log2 M), 0 for M = 1. */
static int ceil_log2(int64_t M)
{
    int L = 0;
    while (((int64_t)1 << L) < M) ++L;
    return L;
}

/* ------------------------------------------------------------------ */
/* Exact inverse-transform fallback in fixed point.                    */
/* F_j = floor(alpha_j * 2^(63-L-E)) with 2^(E-1) <= alpha_max < 2^E.   */
/* Each F_j < 2^(63-L), so S = sum F_j < 2^63.  target = floor(V*S/2^64) */
/* for a 64-bit uniform V; the answer is the least j whose inclusive    */
/* prefix sum exceeds target.                                          */
/* ------------------------------------------------------------------ */
static uint64_t fixed_weight(float a, int shift)
{
    return (uint64_t)ldexpf(a, shift);
}

static uint64_t fixed_sum(const float *a, int64_t stride, int64_t M, int shift)
{
    uint64_t S = 0;
    for (int64_t j = 0; j < M; ++j) S += fixed_weight(a[j * stride], shift);
    return S;
}

static int32_t fallback_pick(const float *a, int64_t stride, int64_t M, int shift,
                             uint64_t S, uint64_t V)
{
    uint64_t target = (uint64_t)(((unsigned __int128)V * S) >> 64);
    uint64_t P = 0;
    for (int64_t j = 0; j < M; ++j) {
        P += fixed_weight(a[j * stride], shift);
        if (P > target) return (int32_t)j;
    }
    return -1; /* unreachable when S > 0 */
}

/* alpha_0 reported from the fixed-point sum: (float)S rounded to nearest even,
 * scaled back by 2^(E-63+L). */
static float fixed_alpha0(uint64_t S, int shift)
{
    return ldexpf((float)S, -shift);
}

/* Scan: validity and exact maximum.  Returns 0 ok, -2 invalid. */
static int scan_max(const float *a, int64_t stride, int64_t M, float *amax)
{
    float m = 0.0f;
    for (int64_t j = 0; j < M; ++j) {
        float x = a[j * stride];
        if (!(x >= 0.0f) || x == INFINITY) return -2;
        if (x > m) m = x;
    }
    *amax = m;
    return 0;
}

/* flags */
#define ORC_DEBUG_CHECK_BOUND 1u

/* ------------------------------------------------------------------ */
/* Uniform-proposal AR, one instance.                                   */
/* ------------------------------------------------------------------ */
static int32_t select_uniform_one(const float *a, int64_t stride, int64_t M,
                                  const float *bound, uint32_t flags, uint32_t k,
                                  uint64_t seed, uint64_t step, uint32_t tag,
                                  uint32_t t_max, float *alpha0, uint32_t *trials)
{
    float amax = 0.0f, env;
    int have_max = 0;
    if (trials) *trials = 0;
    if (bound == NULL || (flags & ORC_DEBUG_CHECK_BOUND) || alpha0 != NULL) {
        if (scan_max(a, stride, M, &amax) != 0) {
            if (alpha0) *alpha0 = NAN;
            return -2;
        }
        have_max = 1;
    }
    if (bound != NULL) {
        env = *bound;
        if (env != env || env < 0.0f || env == INFINITY) {
            if (alpha0) *alpha0 = NAN;
            return -2;
        }
        if (have_max && (flags & ORC_DEBUG_CHECK_BOUND) && amax > env) {
            if (alpha0) *alpha0 = NAN;
            return -3;
        }
        if (env == 0.0f) {
            if (alpha0) *alpha0 = 0.0f;
            return -1;
        }
    } else {
        env = amax;
    }
    int L = ceil_log2(M);
    if (have_max) {
        if (amax == 0.0f) {
            if (alpha0) *alpha0 = 0.0f;
            return -1;
        }
        if (alpha0) {
            int E;
            frexpf(amax, &E);
            *alpha0 = fixed_alpha0(fixed_sum(a, stride, M, 63 - L - E), 63 - L - E);
        }
    }

    /* The sequential rule: trials t = 0, 1, ...; the first accepted wins. */
    uint32_t lemire_floor = (uint32_t)(0u - (uint32_t)M) % (uint32_t)M; /* 2^32 mod M */
    for (uint32_t t = 0; t < t_max; ++t) {
        uint32_t cw, uw;
        trial_words(seed, t, k, step, tag, &cw, &uw);
        uint64_t m = (uint64_t)cw * (uint64_t)M;
        if ((uint32_t)m < lemire_floor) continue;  /* candidate draw rejected */
        int64_t j = (int64_t)(m >> 32);
        double u = grid_u(uw);
        if (u * (double)env < (double)a[j * stride]) {
            if (trials) *trials = t + 1;
            return (int32_t)j;
        }
    }

    /* Fallback: exact inverse transform on the true maximum. */
    if (!have_max) {
        if (scan_max(a, stride, M, &amax) != 0) return -2;
        if (amax == 0.0f) return -1;
    }
    int E;
    frexpf(amax, &E);
    int shift = 63 - L - E;
    uint64_t S = fixed_sum(a, stride, M, shift);
    uint32_t w[4];
    draw(seed, FALLBACK_WORD, k, step, tag, w);
    uint64_t V = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    if (trials) *trials = t_max + 1;
    return fallback_pick(a, stride, M, shift, S, V);
}

/* Dense batch.  layout 0 (AoS): alpha[k*ld + j] (ld = 0 broadcasts one vector);
 * layout 1 (SoA): alpha[j*ld + k].  bound: NULL or K per-instance bounds. */
int orc_select_uniform(const float *alpha, int64_t M, int64_t K, int64_t ld, int layout,
                       const float *bound, uint64_t seed, uint64_t step, uint32_t t_max,
                       uint32_t flags, int32_t *index, float *alpha0, uint32_t *trials,
                       int threads)
{
    if (M < 1 || K < 0 || (layout != 0 && layout != 1)) return -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 16) if (threads != 1)
#endif
    for (int64_t k = 0; k < K; ++k) {
        const float *a;
        int64_t stride;
        if (layout == 0) { a = alpha + k * ld; stride = 1; }
        else             { a = alpha + k;      stride = ld; }
        index[k] = select_uniform_one(a, stride, M, bound ? bound + k : NULL, flags,
                                      (uint32_t)k, seed, step, 0u, t_max,
                                      alpha0 ? alpha0 + k : NULL,
                                      trials ? trials + k : NULL);
    }
    return 0;
}

/* Ragged batch: instance k is alpha[offsets[k] .. offsets[k+1]).  With ids,
 * only instances ids[0..n) are selected (output i for instance ids[i]);
 * otherwise all n instances in order. */
int orc_select_ragged(const float *alpha, const int64_t *offsets, int64_t n,
                      const int64_t *ids, uint64_t seed, uint64_t step, uint32_t t_max,
                      int32_t *index, float *alpha0, uint32_t *trials, int threads)
{
    if (n < 0) return -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) if (threads != 1)
#endif
    for (int64_t i = 0; i < n; ++i) {
        const int64_t k = ids ? ids[i] : i;
        int64_t M = offsets[k + 1] - offsets[k];
        if (M < 1) {
            index[i] = M == 0 ? -1 : -2;
            if (alpha0) alpha0[i] = M == 0 ? 0.0f : NAN;
            if (trials) trials[i] = 0;
            continue;
        }
        index[i] = select_uniform_one(alpha + offsets[k], 1, M, NULL, 0u, (uint32_t)k,
                                      seed, step, 0u, t_max,
                                      alpha0 ? alpha0 + i : NULL,
                                      trials ? trials + i : NULL);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* AR with an integer proposal Q (acceptance probability               */
/* alpha_j / (c+ * Q_j)); the candidate is drawn from Q by the inverse  */
/* transform of its exact integer prefix sums.                          */
/* -4: the proposal is unusable (sum Q >= 2^32, or Q_j = 0 where        */
/* alpha_j > 0).                                                         */
/* ------------------------------------------------------------------ */
/* cbound (nullable): a bound C >= max_j alpha_j / Q_j used in place of the
 * exact c (the bound-maintenance mode of the SSA run). */
static int32_t select_proposal_one(const float *a, const uint32_t *q, int64_t M,
                                   uint32_t k, uint64_t seed, uint64_t step,
                                   uint32_t t_max, uint32_t *trials, uint32_t *prefix,
                                   const double *cbound)
{
    float amax;
    if (trials) *trials = 0;
    if (scan_max(a, 1, M, &amax) != 0) return -2;
    if (amax == 0.0f) return -1;
    uint64_t SQ = 0;
    double c = 0.0;
    for (int64_t j = 0; j < M; ++j) {
        if (a[j] > 0.0f && q[j] == 0u) return -4;
        SQ += q[j];
        prefix[j] = (uint32_t)SQ;
        if (a[j] > 0.0f) {
            double r = (double)a[j] / (double)q[j];
            if (r > c) c = r;
        }
    }
    if (SQ >= ((uint64_t)1 << 32)) return -4;
    if (cbound) c = *cbound;
    /* c+ >= alpha_j / Q_j for every j, so no acceptance probability saturates */
    double cplus = nextafter(c, INFINITY);
    uint32_t sq = (uint32_t)SQ;
    uint32_t lemire_floor = (0u - sq) % sq;
    for (uint32_t t = 0; t < t_max; ++t) {
        uint32_t cw, uw;
        trial_words(seed, t, k, step, 1u, &cw, &uw);
        uint64_t m = (uint64_t)cw * (uint64_t)sq;
        if ((uint32_t)m < lemire_floor) continue;
        uint32_t V = (uint32_t)(m >> 32);
        /* least j with prefix[j] > V: binary search over the prefix sums */
        int64_t lo = 0, hi = M - 1;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (prefix[mid] > V) hi = mid; else lo = mid + 1;
        }
        int64_t j = lo;
        double u = grid_u(uw);
        double uc = u * cplus;
        if (uc * (double)q[j] < (double)a[j]) {
            if (trials) *trials = t + 1;
            return (int32_t)j;
        }
    }
    int L = ceil_log2(M);
    int E;
    frexpf(amax, &E);
    int shift = 63 - L - E;
    uint64_t S = fixed_sum(a, 1, M, shift);
    uint32_t w[4];
    draw(seed, FALLBACK_WORD, k, step, 1u, w);
    uint64_t V = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
    if (trials) *trials = t_max + 1;
    return fallback_pick(a, 1, M, shift, S, V);
}

/* alpha[k*lda + j], Q[k*ldq + j]. */
int orc_select_proposal(const float *alpha, const uint32_t *Q, int64_t M, int64_t K,
                        int64_t lda, int64_t ldq, uint64_t seed, uint64_t step,
                        uint32_t t_max, int32_t *index, uint32_t *trials, int threads)
{
    if (M < 1 || K < 0) return -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel if (threads != 1)
#endif
    {
        uint32_t *prefix = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)M);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t k = 0; k < K; ++k) {
            index[k] = select_proposal_one(alpha + k * lda, Q + k * ldq, M, (uint32_t)k,
                                           seed, step, t_max,
                                           trials ? trials + k : NULL, prefix, NULL);
        }
        free(prefix);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Mass-action propensities and the SSA jump chain (state sequence of   */
/* the direct method; the holding times do not change the sequence).    */
/* ------------------------------------------------------------------ */
static float mass_action(const int32_t *x, int32_t r0, int32_t r1, float rate)
{
    int64_t h;
    if (r1 < 0)        h = x[r0];
    else if (r1 == r0) h = (int64_t)x[r0] * (x[r0] - 1) / 2;
    else               h = (int64_t)x[r0] * x[r1];
    return rate * (float)h;
}

/* alpha[r*M + j] for states X[r*N + i]. */
void orc_propensities(const int32_t *X, int64_t R, int64_t N, int64_t M,
                      const int32_t *r0, const int32_t *r1, const float *rate,
                      float *alpha)
{
    (void)N;
    for (int64_t r = 0; r < R; ++r)
        for (int64_t j = 0; j < M; ++j)
            alpha[r * M + j] = mass_action(X + r * N, r0[j], r1[j], rate[j]);
}

/* Run `steps` jump-chain steps for R realizations in place on X[r*N + i].
 * Step i of realization r selects with uniform AR (tag 2, instance r,
 * step step0 + i); a selection < 0 (nothing can fire) leaves the state.
 * When rec_X is non-NULL, the state before each step i >= rec_from is
 * written to rec_X[((i - rec_from) * R + r) * N + ...]. */
int orc_ssa_chain(int32_t *X, int64_t R, int64_t N, int64_t M,
                  const int32_t *r0, const int32_t *r1, const int32_t *p0,
                  const int32_t *p1, const float *rate, uint64_t seed, uint64_t step0,
                  int64_t steps, uint32_t t_max, int64_t rec_from, int32_t *rec_X,
                  int32_t *fired, int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel if (threads != 1)
#endif
    {
        float *a = (float *)malloc(sizeof(float) * (size_t)M);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t r = 0; r < R; ++r) {
            int32_t *x = X + r * N;
            for (int64_t i = 0; i < steps; ++i) {
                if (rec_X && i >= rec_from)
                    memcpy(rec_X + ((i - rec_from) * R + r) * N, x, sizeof(int32_t) * (size_t)N);
                for (int64_t j = 0; j < M; ++j)
                    a[j] = mass_action(x, r0[j], r1[j], rate[j]);
                int32_t j = select_uniform_one(a, 1, M, NULL, 0u, (uint32_t)r, seed,
                                               step0 + (uint64_t)i, 2u, t_max, NULL, NULL);
                if (fired) fired[i * R + r] = j;
                if (j < 0) continue;
                x[r0[j]] -= 1;
                if (r1[j] >= 0) x[r1[j]] -= 1;
                x[p0[j]] += 1;
                if (p1[j] >= 0) x[p1[j]] += 1;
            }
        }
        free(a);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* ln of the time step: P. T. P. Tang, "Table-driven implementation of   */
/* the logarithm function in IEEE floating-point arithmetic", ACM TOMS   */
/* 16(4), 1990, in this variant:                                        */
/*   u = m 2^e with m in [0.75, 1.5);                                   */
/*   c = i / 128, the breakpoint nearest m (ties to even), i in 96..192; */
/*   r = (m - c) * fl(1 / c), where m - c is exact;                     */
/*   log1p(r) by its Taylor polynomial of degree 7, r (1 - r/2 + ... +   */
/*   r^6/7), the bracket by Horner's rule from 1/7 down with fused      */
/*   multiply-adds, then one product with r;                            */
/*   ln u = fma(e, fl(ln 2), fl(ln c)) + log1p(r).                      */
/* fl(ln c) and fl(1 / c) are the rounded values (libm log of the exact  */
/* i / 128, one IEEE division).  |r| <= 2^-8 / 0.75, so the first       */
/* omitted term is below 2^-56 of log1p(r).                             */
/* ------------------------------------------------------------------ */
static double ln_c[193], inv_c[193];   /* entries 96..192 */
static int ln_ready;

static void ln_table_init(void)
{
    if (ln_ready) return;
    for (int i = 96; i <= 192; ++i) {
        ln_c[i] = log((double)i / 128.0);
        inv_c[i] = 128.0 / (double)i;
    }
    ln_ready = 1;
}

/* -ln u for u = (w + 1/2) 2^-32, the time step's uniform. */
static double neg_ln_uniform(uint32_t w)
{
    static const double coef[7] = {1.0 / 7.0, -1.0 / 6.0, 1.0 / 5.0, -1.0 / 4.0,
                                   1.0 / 3.0, -1.0 / 2.0, 1.0};
    const double u = ((double)w + 0.5) * 0x1p-32;
    int e;
    double m = frexp(u, &e);                  /* u = m 2^e, m in [0.5, 1) */
    if (m < 0.75) {
        m *= 2.0;
        e -= 1;
    }
    const int i = (int)nearbyint(m * 128.0);
    const double r = (m - (double)i / 128.0) * inv_c[i];
    double p = coef[0];
    for (int k = 1; k < 7; ++k) p = fma(p, r, coef[k]);
    return -(fma((double)e, M_LN2, ln_c[i]) + p * r);
}

double orc_neg_ln_uniform(uint32_t w)
{
    ln_table_init();
    return neg_ln_uniform(w);
}

/* ------------------------------------------------------------------ */
/* alpha_0 of the time step.  With a scale exponent E (2^(E-1) <= a      */
/* maximum of the propensities < 2^E, chosen below) and                 */
/* sh = 127 - L - E, each finite positive alpha_j contributes           */
/* F_j = floor(alpha_j 2^sh) < 2^(127-L); S = sum F_j < 2^127 is exact   */
/* in an unsigned 128-bit integer, and alpha_0 = fl64(S) 2^-sh (one     */
/* rounding, to nearest even).  Every alpha_j >= 2^(E-103+L) is a whole */
/* multiple of 2^-sh, so when the positive propensities lie within      */
/* 104 - L binades of 2^E, alpha_0 is their exact sum rounded once;     */
/* below that, the parts under 2^-sh are dropped (M 2^-sh at most).     */
/* The run keeps S >= 2^(95-L) (alpha_0 >= 2^(E-32)), so the dropped     */
/* parts stay below 2^(2L-95) of alpha_0.                               */
/* ------------------------------------------------------------------ */
#define NO_SCALE (-100000)

static int exponent_above(float a)
{
    int e;
    (void)frexpf(a, &e);
    return e;
}

/* floor(a 2^sh) for finite a > 0: a = f 2^e with f in [0.5, 1), so
 * a = n 2^(e-24) with the integer n = f 2^24 < 2^24, and the floor is n
 * shifted by e - 24 + sh (right shifts drop the fraction). */
static unsigned __int128 wide_weight(float a, int sh)
{
    int e;
    const float f = frexpf(a, &e);
    const unsigned __int128 n = (uint32_t)ldexpf(f, 24);
    const int s = e - 24 + sh;
    if (s >= 0) return n << s;
    return s > -32 ? n >> -s : 0;
}

static unsigned __int128 wide_sum(const float *a, int64_t M, int E)
{
    const int sh = 127 - ceil_log2(M) - E;
    unsigned __int128 S = 0;
    for (int64_t j = 0; j < M; ++j)
        if (a[j] > 0.0f && a[j] < INFINITY) S += wide_weight(a[j], sh);
    return S;
}

static double wide_alpha0(const float *a, int64_t M, int E)
{
    return ldexp((double)wide_sum(a, M, E), -(127 - ceil_log2(M) - E));
}

double orc_wide_alpha0(const float *a, int64_t M, int E)
{
    return wide_alpha0(a, M, E);
}

/* ------------------------------------------------------------------ */
/* Full SSA run (direct method, section "The Stochastic Simulation      */
/* Algorithm"): each step recomputes every propensity from the state,   */
/* selects the next reaction, advances the time by                      */
/* tau = ln(1/u) / alpha_0 and applies the stoichiometry.  u comes from */
/* Philox block 0xFFFFFFFE of the tag-2 stream (instance id, step s),    */
/* word 0, as (w + 1/2) 2^-32 in (0, 1); -ln u is neg_ln_uniform and    */
/* alpha_0 is wide_alpha0 with the scale exponent E: at the call's first */
/* step and at steps with s mod p = 0 (the exact steps, below), E is    */
/* that of alpha_max (none when a propensity is invalid or all are      */
/* zero); between them E stays while every valid propensity is below    */
/* 2^E and is dropped once one reaches it; a step that fires with no E, */
/* or with S < 2^(95-L) at E (alpha_0 fell 32 binades below 2^E), takes */
/* E from its own alpha_max.  An invalid propensity records -2          */
/* and every propensity zero records -1; state and time then stay.      */
/*                                                                      */
/* Selection: uniform AR on the tag-2 stream (the jump chain's) with    */
/* the envelope B, or, with a proposal Q, proposal AR on the tag-1       */
/* stream with Q'_j = max(Q_j, qfloor, 1) and the envelope C.  With      */
/* period p, B and C are exact (alpha_max and max_j fl64(alpha_j/Q'_j))  */
/* at the first step of the call and at steps s with s mod p = 0; at    */
/* other steps they are the running maximum of those quantities since   */
/* then (bounds kept from the propensities that change: the dependency  */
/* graph idea the Introduction cites from the Next Reaction Method).    */
/* Any B >= alpha_max and C >= max alpha_j / Q'_j leave the law of each  */
/* step alpha_j / alpha_0; p = 1 (or 0) is exact at every step.          */
/* ids[r] (or r when ids is NULL) is realization r's instance id.       */
/* t[r] is read and advanced in place; times (nullable) receives t after */
/* each step at [i * R + r]; fired (nullable) the selection at [i*R+r]. */
/* ------------------------------------------------------------------ */
#define TAU_BLOCK 0xFFFFFFFEu

static int ssa_run(int32_t *X, int64_t R, int64_t N, int64_t M, const int32_t *r0,
                   const int32_t *r1, const int32_t *p0, const int32_t *p1, const float *rate,
                   const uint32_t *Q, int64_t ldq, uint32_t qfloor, uint32_t period,
                   const uint32_t *ids, uint64_t seed, uint64_t step0, int64_t steps,
                   uint32_t t_max, double *t, double *times, int32_t *fired, int threads)
{
    if (period == 0) period = 1;
    ln_table_init();
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel if (threads != 1)
#endif
    {
        float *a = (float *)malloc(sizeof(float) * (size_t)M);
        uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)M);
        uint32_t *prefix = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)M);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t r = 0; r < R; ++r) {
            int32_t *x = X + r * N;
            const uint32_t id = ids ? ids[r] : (uint32_t)r;
            if (Q) {
                const uint32_t lo = qfloor > 0u ? qfloor : 1u;
                for (int64_t j = 0; j < M; ++j) {
                    const uint32_t v = Q[r * ldq + j];
                    q[j] = v > lo ? v : lo;
                }
            }
            float B = 0.0f;
            double C = 0.0;
            int E = NO_SCALE;
            for (int64_t i = 0; i < steps; ++i) {
                const uint64_t s = step0 + (uint64_t)i;
                const int exact = i == 0 || s % period == 0;
                float vmax = 0.0f;             /* largest valid propensity */
                for (int64_t j = 0; j < M; ++j) {
                    a[j] = mass_action(x, r0[j], r1[j], rate[j]);
                    if (a[j] >= 0.0f && a[j] < INFINITY && a[j] > vmax) vmax = a[j];
                }
                float amax;
                const int ok = scan_max(a, 1, M, &amax) == 0;
                if (exact)
                    E = ok && amax > 0.0f ? exponent_above(amax) : NO_SCALE;
                else if (E != NO_SCALE && (double)vmax >= ldexp(1.0, E))
                    E = NO_SCALE;
                int32_t j;
                if (!ok) {
                    j = -2;
                } else if (amax == 0.0f) {
                    j = -1;
                } else if (Q == NULL) {
                    B = exact || amax > B ? amax : B;
                    j = select_uniform_one(a, 1, M, &B, 0u, id, seed, s, 2u, t_max, NULL, NULL);
                } else {
                    double c = 0.0;
                    for (int64_t jj = 0; jj < M; ++jj)
                        if (a[jj] > 0.0f) {
                            const double v = (double)a[jj] / (double)q[jj];
                            if (v > c) c = v;
                        }
                    C = exact || c > C ? c : C;
                    j = select_proposal_one(a, q, M, id, seed, s, t_max, NULL, prefix, &C);
                }
                if (fired) fired[i * R + r] = j;
                if (j >= 0) {
                    uint32_t w[4];
                    draw(seed, TAU_BLOCK, id, s, 2u, w);
                    const int L = ceil_log2(M);
                    unsigned __int128 S = 0;
                    if (E != NO_SCALE) S = wide_sum(a, M, E);
                    if (E != NO_SCALE && S < (unsigned __int128)1 << (95 - L)) E = NO_SCALE;
                    if (E == NO_SCALE) {
                        E = exponent_above(amax);
                        S = wide_sum(a, M, E);
                    }
                    t[r] += neg_ln_uniform(w[0]) / ldexp((double)S, -(127 - L - E));
                    x[r0[j]] -= 1;
                    if (r1[j] >= 0) x[r1[j]] -= 1;
                    x[p0[j]] += 1;
                    if (p1[j] >= 0) x[p1[j]] += 1;
                }
                if (times) times[i * R + r] = t[r];
            }
        }
        free(a);
        free(q);
        free(prefix);
    }
    return 0;
}

int orc_ssa_run(int32_t *X, int64_t R, int64_t N, int64_t M,
                const int32_t *r0, const int32_t *r1, const int32_t *p0, const int32_t *p1,
                const float *rate, uint32_t period, const uint32_t *ids, uint64_t seed,
                uint64_t step0, int64_t steps, uint32_t t_max, double *t, double *times,
                int32_t *fired, int threads)
{
    return ssa_run(X, R, N, M, r0, r1, p0, p1, rate, NULL, 0, 0u, period, ids, seed, step0,
                   steps, t_max, t, times, fired, threads);
}

/* The run with an integer proposal (the learned proposal refreshed lazily,
 * held fixed for the call; Q is [R][ldq] uint32, realization r's row).  The
 * floor keeps reactions that turn active during the call covered, with a
 * weight the caller sizes against the scale of Q. */
int orc_ssa_run_proposal(int32_t *X, int64_t R, int64_t N, int64_t M,
                         const int32_t *r0, const int32_t *r1, const int32_t *p0,
                         const int32_t *p1, const float *rate, const uint32_t *Q, int64_t ldq,
                         uint32_t qfloor, uint32_t period, const uint32_t *ids, uint64_t seed,
                         uint64_t step0, int64_t steps, uint32_t t_max, double *t,
                         double *times, int32_t *fired, int threads)
{
    return ssa_run(X, R, N, M, r0, r1, p0, p1, rate, Q, ldq, qfloor, period, ids, seed, step0,
                   steps, t_max, t, times, fired, threads);
}

/* ------------------------------------------------------------------ */
/* The paper's own scheme (section "A GPU acceptance-rejection          */
/* algorithm (GPU/AR) for SSA", election and selection steps): every    */
/* reaction j draws u_j in [0, T), is eligible when u_j < D_j (D_j > 0)  */
/* and is rated R_j = u_j / D_j; the eligible reaction with the lowest  */
/* rating is selected, and when none is eligible the election fails    */
/* (the paper returns M + 1; here -5).  T = w * alpha_max (the paper's  */
/* T_w).  Reaction j takes word j mod 4 of Philox block j / 4 of the     */
/* tag-3 stream (instance k, step s): u_j = w_j 2^-32 T in binary64.     */
/* The pseudo-code's default rating 10 T for a non-eligible reaction    */
/* can undercut real ratings when T < 0.1; here a non-eligible reaction */
/* never wins.  Equal ratings go to the least index.  The law is not    */
/* alpha_j / alpha_0 (see oracle/laws.py, paper_law).                   */
/* ------------------------------------------------------------------ */
static int32_t select_paper_one(const float *a, int64_t stride, int64_t M, double w,
                                uint32_t k, uint64_t seed, uint64_t step)
{
    float amax;
    if (scan_max(a, stride, M, &amax) != 0) return -2;
    if (amax == 0.0f) return -1;
    const double T = w * (double)amax;
    int32_t best = -5;
    double best_r = 0.0;
    uint32_t words[4];
    for (int64_t j = 0; j < M; ++j) {
        if ((j & 3) == 0) draw(seed, (uint32_t)(j >> 2), k, step, 3u, words);
        const double u = grid_u(words[j & 3]) * T;
        const double d = (double)a[j * stride];
        if (d > 0.0 && u < d) {
            const double r = u / d;
            if (best < 0 || r < best_r) {
                best = (int32_t)j;
                best_r = r;
            }
        }
    }
    return best;
}

int orc_select_paper(const float *alpha, int64_t M, int64_t K, int64_t ld, double w,
                     uint64_t seed, uint64_t step, int32_t *index, int threads)
{
    if (M < 1 || K < 0 || (ld != 0 && ld < M) || !(w > 0.0)) return -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static) if (threads != 1)
#endif
    for (int64_t k = 0; k < K; ++k)
        index[k] = select_paper_one(alpha + k * ld, 1, M, w, (uint32_t)k, seed, step);
    return 0;
}

/* Uniform AR for n instances given as rows alpha[i*M + j] whose instance ids
 * (Philox stream) are ids[i]: the same selection as orc_select_uniform gives
 * instance ids[i] of a larger batch, for checking sampled instances. */
int orc_select_ids(const float *alpha, int64_t M, int64_t n, const uint32_t *ids,
                   uint64_t seed, uint64_t step, uint32_t t_max, int32_t *index,
                   float *alpha0, uint32_t *trials, int threads)
{
    if (M < 1 || n < 0 || !ids) return -1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1) if (threads != 1)
#endif
    for (int64_t i = 0; i < n; ++i)
        index[i] = select_uniform_one(alpha + i * M, 1, M, NULL, 0u, ids[i], seed, step, 0u,
                                      t_max, alpha0 ? alpha0 + i : NULL, trials ? trials + i : NULL);
    return 0;
}
