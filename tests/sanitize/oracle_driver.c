/* Host sanitizer driver for the CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Built together with oracle/arsel_oracle.c by gcc with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py) and run on small
 * inputs that reach every entry point and their edge cases: broadcast, AoS,
 * SoA and bounded batches, forced fallbacks, empty and invalid instances,
 * proposals with uncovered support, the SSA chain and runs (with and without a
 * proposal, exact and maintained envelopes), the paper's scheme and selection
 * by instance id.  Exit status 0 and no sanitizer report is a pass. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int orc_select_uniform(const float *alpha, int64_t M, int64_t K, int64_t ld, int layout,
                       const float *bound, uint64_t seed, uint64_t step, uint32_t t_max,
                       uint32_t flags, int32_t *index, float *alpha0, uint32_t *trials,
                       int threads);
int orc_select_ragged(const float *alpha, const int64_t *offsets, int64_t n, const int64_t *ids,
                      uint64_t seed, uint64_t step, uint32_t t_max, int32_t *index,
                      float *alpha0, uint32_t *trials, int threads);
int orc_select_proposal(const float *alpha, const uint32_t *Q, int64_t M, int64_t K,
                        int64_t lda, int64_t ldq, uint64_t seed, uint64_t step,
                        uint32_t t_max, int32_t *index, uint32_t *trials, int threads);
void orc_propensities(const int32_t *X, int64_t R, int64_t N, int64_t M, const int32_t *r0,
                      const int32_t *r1, const float *rate, float *alpha);
int orc_ssa_chain(int32_t *X, int64_t R, int64_t N, int64_t M, const int32_t *r0,
                  const int32_t *r1, const int32_t *p0, const int32_t *p1, const float *rate,
                  uint64_t seed, uint64_t step0, int64_t steps, uint32_t t_max,
                  int64_t rec_from, int32_t *rec_X, int32_t *fired, int threads);
int orc_ssa_run(int32_t *X, int64_t R, int64_t N, int64_t M, const int32_t *r0,
                const int32_t *r1, const int32_t *p0, const int32_t *p1, const float *rate,
                uint32_t period, const uint32_t *ids, uint64_t seed, uint64_t step0,
                int64_t steps, uint32_t t_max, double *t, double *times, int32_t *fired,
                int threads);
int orc_ssa_run_proposal(int32_t *X, int64_t R, int64_t N, int64_t M, const int32_t *r0,
                         const int32_t *r1, const int32_t *p0, const int32_t *p1,
                         const float *rate, const uint32_t *Q, int64_t ldq, uint32_t qfloor,
                         uint32_t period, const uint32_t *ids, uint64_t seed, uint64_t step0,
                         int64_t steps, uint32_t t_max, double *t, double *times,
                         int32_t *fired, int threads);
double orc_neg_ln_uniform(uint32_t w);
double orc_wide_alpha0(const float *a, int64_t M, int E);
int orc_select_paper(const float *alpha, int64_t M, int64_t K, int64_t ld, double w,
                     uint64_t seed, uint64_t step, int32_t *index, int threads);
int orc_select_ids(const float *alpha, int64_t M, int64_t n, const uint32_t *ids,
                   uint64_t seed, uint64_t step, uint32_t t_max, int32_t *index,
                   float *alpha0, uint32_t *trials, int threads);

static uint64_t lcg = 12345;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * 0x1p-53;
}

static int fails = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

static void dense(void)
{
    enum { M = 37, K = 21 };
    float *a = malloc(sizeof(float) * M * K);      /* exact sizes: overruns are reported */
    float *bound = malloc(sizeof(float) * K);
    int32_t *idx = malloc(sizeof(int32_t) * K);
    float *a0 = malloc(sizeof(float) * K);
    uint32_t *tr = malloc(sizeof(uint32_t) * K);
    for (int i = 0; i < M * K; ++i) a[i] = unif() < 0.3 ? 0.0f : (float)(-log(1.0 - unif()));
    for (int j = 0; j < M; ++j) a[3 * M + j] = 0.0f;          /* instance 3: all zero (AoS) */
    a[5 * M + 7] = NAN;                                        /* instance 5: invalid (AoS) */
    a[6 * M + 2] = -1.0f;
    a[7 * M + 1] = INFINITY;
    a[8 * M + 4] = 1e-45f;                                     /* subnormal */
    for (int k = 0; k < K; ++k) bound[k] = 1e3f;
    bound[2] = 0.0f;
    bound[4] = NAN;
    for (uint32_t t_max = 0; t_max <= 4096; t_max = t_max ? t_max * 8 : 1) {
        CHECK(orc_select_uniform(a, M, K, M, 0, NULL, 1, t_max, t_max, 0, idx, a0, tr, 1) == 0);
        CHECK(idx[3] == -1 && idx[5] == -2 && idx[6] == -2 && idx[7] == -2);
        CHECK(orc_select_uniform(a, M, K, K, 1, NULL, 1, t_max, t_max, 0, idx, a0, tr, 1) == 0);
        CHECK(orc_select_uniform(a, M, K, 0, 0, NULL, 2, 0, t_max, 0, idx, NULL, NULL, 1) == 0);
        CHECK(orc_select_uniform(a, M, K, M, 0, bound, 3, 0, t_max, 1, idx, a0, tr, 1) == 0);
        CHECK(orc_select_uniform(a, M, K, M, 0, bound, 3, 0, t_max, 0, idx, NULL, tr, 1) == 0);
    }
    CHECK(orc_select_uniform(a, 1, K, 1, 0, NULL, 1, 0, 4096, 0, idx, a0, tr, 1) == 0);
    CHECK(orc_select_uniform(a, M, 0, M, 0, NULL, 1, 0, 4096, 0, idx, a0, tr, 1) == 0);
    CHECK(orc_select_uniform(a, 0, K, M, 0, NULL, 1, 0, 4096, 0, idx, a0, tr, 1) != 0);
    uint32_t ids[K];
    for (int i = 0; i < K; ++i) ids[i] = 1000u * (uint32_t)i + 7u;
    CHECK(orc_select_ids(a, M, K, ids, 4, 5, 4096, idx, a0, tr, 1) == 0);
    CHECK(orc_select_paper(a, M, K, M, 1.0, 1, 0, idx, 1) == 0);
    CHECK(orc_select_paper(a, M, K, 0, 2.0, 1, 0, idx, 1) == 0);
    free(a); free(bound); free(idx); free(a0); free(tr);
}

static void ragged(void)
{
    enum { K = 9 };
    const int64_t sizes[K] = {0, 1, 5, 0, 700, 64, 3, 2000, 0};
    int64_t off[K + 1];
    off[0] = 0;
    for (int k = 0; k < K; ++k) off[k + 1] = off[k] + sizes[k];
    float *a = malloc(sizeof(float) * (size_t)off[K]);
    for (int64_t i = 0; i < off[K]; ++i) a[i] = (float)exp(3.0 * (unif() - 0.5) * 4.0);
    a[off[2] + 1] = NAN;
    int32_t idx[K];
    float a0[K];
    uint32_t tr[K];
    const int64_t ids[3] = {8, 4, 0};
    for (uint32_t t_max = 0; t_max <= 4096; t_max = t_max ? t_max * 16 : 1) {
        CHECK(orc_select_ragged(a, off, K, NULL, 9, t_max, t_max, idx, a0, tr, 1) == 0);
        CHECK(idx[0] == -1 && idx[2] == -2 && idx[1] == 0);
        CHECK(orc_select_ragged(a, off, 3, ids, 9, 1, t_max, idx, NULL, NULL, 1) == 0);
    }
    free(a);
}

static void proposal(void)
{
    enum { M = 29, K = 6 };
    float *a = malloc(sizeof(float) * M * K);
    uint32_t *Q = malloc(sizeof(uint32_t) * M * K);
    int32_t idx[K];
    uint32_t tr[K];
    for (int i = 0; i < M * K; ++i) {
        a[i] = unif() < 0.25 ? 0.0f : (float)unif();
        Q[i] = a[i] > 0.0f ? 1u + (uint32_t)(unif() * 1000) : 0u;
    }
    Q[1 * M + 3] = 0; a[1 * M + 3] = 1.0f;                     /* uncovered support: -4 */
    Q[2 * M + 0] = 0xFFFFFFFFu; Q[2 * M + 1] = 9;              /* sum >= 2^32 */
    for (int j = 0; j < M; ++j) a[3 * M + j] = 0.0f;
    for (uint32_t t_max = 0; t_max <= 4096; t_max = t_max ? t_max * 8 : 1) {
        CHECK(orc_select_proposal(a, Q, M, K, M, M, 5, t_max, t_max, idx, tr, 1) == 0);
        CHECK(idx[1] == -4 && idx[3] == -1);
        CHECK(orc_select_proposal(a, Q, M, K, 0, 0, 5, t_max, t_max, idx, NULL, 1) == 0);
    }
    free(a); free(Q);
}

static void ssa(void)
{
    enum { N = 6, M = 8, R = 5, STEPS = 300 };
    const int32_t r0[M] = {0, 1, 2, 3, 4, 5, 0, 2};
    const int32_t r1[M] = {-1, 2, -1, 3, -1, 0, 0, -1};
    const int32_t p0[M] = {1, 3, 4, 5, 0, 2, 4, 1};
    const int32_t p1[M] = {-1, 0, -1, 1, -1, 3, 5, -1};
    const float rate[M] = {1.0f, 0.01f, 0.5f, 0.002f, 2.0f, 0.03f, 0.001f, 0.7f};
    int32_t *X = malloc(sizeof(int32_t) * N * R);
    int32_t *X0 = malloc(sizeof(int32_t) * N * R);
    for (int i = 0; i < N * R; ++i) X0[i] = (int32_t)(unif() * 60);
    for (int i = 0; i < N; ++i) X0[4 * N + i] = 0;              /* realization 4 cannot fire */
    float *alpha = malloc(sizeof(float) * M * R);
    orc_propensities(X0, R, N, M, r0, r1, rate, alpha);
    int32_t *rec = malloc(sizeof(int32_t) * (STEPS - 10) * R * N);
    int32_t *fired = malloc(sizeof(int32_t) * STEPS * R);
    double *t = malloc(sizeof(double) * R);
    double *times = malloc(sizeof(double) * STEPS * R);
    uint32_t *Q = malloc(sizeof(uint32_t) * M * R);
    for (int i = 0; i < M * R; ++i) Q[i] = 1u + (uint32_t)(unif() * 100);
    uint32_t ids[R];
    for (int r = 0; r < R; ++r) ids[r] = 100u + 3u * (uint32_t)r;
    memcpy(X, X0, sizeof(int32_t) * N * R);
    CHECK(orc_ssa_chain(X, R, N, M, r0, r1, p0, p1, rate, 3, 0, STEPS, 4096, 10, rec, fired, 1) == 0);
    for (uint32_t period = 0; period <= 64; period = period ? period * 8 : 1) {
        for (int pass = 0; pass < 2; ++pass) {
            memcpy(X, X0, sizeof(int32_t) * N * R);
            for (int r = 0; r < R; ++r) t[r] = 0.0;
            const uint32_t *idp = pass ? ids : NULL;
            CHECK(orc_ssa_run(X, R, N, M, r0, r1, p0, p1, rate, period, idp, 7, 0, STEPS, 4096,
                              t, times, fired, 1) == 0);
            memcpy(X, X0, sizeof(int32_t) * N * R);
            CHECK(orc_ssa_run_proposal(X, R, N, M, r0, r1, p0, p1, rate, Q, M, 5u, period, idp, 7,
                                       0, STEPS, pass ? 3u : 4096u, t, times, fired, 1) == 0);
            CHECK(fired[STEPS * R - 1] == -1);                  /* realization 4 */
        }
    }
    free(X); free(X0); free(alpha); free(rec); free(fired); free(t); free(times); free(Q);
}

/* the time step's pieces at the ends of their ranges: u = 2^-33 and
 * 1 - 2^-33; alpha_0 of subnormals, of FLT_MAX entries, and under a scale
 * far above the values (most weights drop to zero) */
static void time_step(void)
{
    CHECK(orc_neg_ln_uniform(0u) > 22.8 && orc_neg_ln_uniform(0u) < 22.9);
    CHECK(orc_neg_ln_uniform(0xFFFFFFFFu) > 0.0 && orc_neg_ln_uniform(0xFFFFFFFFu) < 1e-9);
    const float sub[4] = {1e-45f, 3e-44f, 0.0f, 7e-40f};
    CHECK(orc_wide_alpha0(sub, 4, -129) > 0.0);
    float big[1000];
    for (int i = 0; i < 1000; ++i) big[i] = 3.4028234e38f;
    CHECK(orc_wide_alpha0(big, 1000, 128) > 3.4e41);
    const float spread[5] = {1e30f, 1e-30f, 1e-40f, -1.0f, 5.0f};
    CHECK(orc_wide_alpha0(spread, 5, 100) > 9.9e29);
    CHECK(orc_wide_alpha0(spread, 5, 127) > 9.9e29);
}

int main(void)
{
    uint32_t out[4];
    const uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0};
    orc_philox4x32_10(ctr, key, out);
    CHECK(out[0] == 0x6627e8d5u);      /* Salmon et al. (SC'11) known-answer vector */
    dense();
    ragged();
    proposal();
    ssa();
    time_step();
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("sanitized oracle run ok\n");
    return 0;
}
