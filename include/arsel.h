/*
 * arsel -- batched acceptance-rejection selection of the next reaction to
 * occur in Gillespie's SSA, for AMD Instinct MI355X (gfx950).
 *
 * Method: Neri & Mestivier, arXiv:1404.0027.  For each of K propensity
 * vectors alpha[0..M) the library returns one reaction index j with
 * probability alpha_j / alpha_0 (alpha_0 = sum_j alpha_j), the selection law
 * of the direct method (section "The Stochastic Simulation Algorithm"),
 * reached by the acceptance-rejection rule of section "A GPU
 * acceptance-rejection algorithm (GPU/AR) for SSA": draw j uniformly and u
 * uniformly in [0,1), accept when u * alpha_max < alpha_j, else draw again.
 *
 * Random stream.  Counter-based Philox4x32-10 keyed by the 64-bit seed.
 * Trial t of instance k at step s uses the block with counter
 * (t/2, k, s mod 2^32, (s >> 32) ^ (tag << 28)); even t takes words (0,1),
 * odd t words (2,3).  The first word of a trial gives the candidate by
 * Lemire's multiply-shift (the 2^32 mod M lowest products are rejected so
 * candidates are exactly uniform), the second gives u = w * 2^-32; the test
 * u * alpha_max < alpha_j is made in binary64.  The answer is the accepted
 * trial with the least t, so it does not depend on how many trials the GPU
 * runs at once.  When t_max trials all reject, the inverse transform of
 * the direct method picks j in exact 64-bit fixed point with the block
 * (0xFFFFFFFF, k, ...): F_j = floor(alpha_j 2^(63-L-E)), L = ceil(log2 M),
 * 2^(E-1) <= alpha_max < 2^E; V = word0 | word1 << 32; j is the least index
 * whose inclusive prefix of F exceeds floor(V * sum F / 2^64).
 * Tags: 0 uniform selection, 1 proposal selection, 2 SSA data generation.
 *
 * Conventions for every entry point.
 *  - Array pointers are DEVICE pointers owned by the caller; the library never
 *    frees them and keeps none of them after the call returns.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    null stream); no call synchronises the device.
 *  - A negative return value is an argument error detected on the host
 *    before anything is launched, or a launch failure (ARSEL_ERR_HIP).
 *  - Per-instance outcomes are reported in `index`: >= 0 the selected
 *    reaction; -1 every propensity is zero (nothing can fire; the paper
 *    returns an out-of-range index in that case); -2 a propensity is NaN,
 *    negative or +inf; -3 a supplied bound is below the true maximum (only
 *    with ARSEL_DEBUG_CHECK_BOUND); -4 an unusable proposal.
 *  - One context per host thread; calls on one context are not thread-safe.
 */
#ifndef ARSEL_H
#define ARSEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct arsel_ctx arsel_ctx;

enum {
    ARSEL_OK = 0,
    ARSEL_ERR_NULL = -1,        /* a required pointer is NULL */
    ARSEL_ERR_SIZE = -2,        /* M < 1, K < 0, or a size beyond the 32-bit index range */
    ARSEL_ERR_LAYOUT = -3,      /* layout is neither ARSEL_AOS nor ARSEL_SOA */
    ARSEL_ERR_LD = -4,          /* leading dimension too small for the layout */
    ARSEL_ERR_HIP = -5,         /* a HIP call or kernel launch failed */
    ARSEL_ERR_DEVICE = -6,      /* bad device id, or the device is not gfx950 */
    ARSEL_ERR_ALLOC = -7,       /* host or device allocation failed */
    ARSEL_ERR_ARG = -8          /* another invalid argument (named by arsel_strerror) */
};

enum { ARSEL_AOS = 0, ARSEL_SOA = 1 };

/* flags */
#define ARSEL_DEBUG_CHECK_BOUND 1u   /* scan alpha even with a supplied bound; -3 if bound < max */

/* Create a context on HIP device `device` (makes it current while creating).
 * The context holds device properties, a small device scratch area and the
 * schedule table used by arsel_select_ragged.  Returns ARSEL_OK or an error. */
int arsel_create(arsel_ctx **out, int device);

/* Free the context and its device scratch.  NULL is accepted. */
int arsel_destroy(arsel_ctx *ctx);

/* Text for an error code (static storage). */
const char *arsel_strerror(int code);

/*
 * Dense batch: K instances with M reactions each (section "Results /
 * Implementation": propensities of realization k stored as D[k*M + j]).
 *   layout ARSEL_AOS: alpha[k*ld + j]; ld == 0 broadcasts one vector to all K
 *                     instances (packed rounds, see arsel_set_trial_lanes);
 *                     otherwise ld >= M.
 *   layout ARSEL_SOA: alpha[j*ld + k], ld >= K (coalesced across instances).
 *   bound:   NULL -> alpha_max is computed per instance (exact maximum);
 *            else K per-instance bounds B_k >= max_j alpha_j used in place of
 *            alpha_max (any such bound keeps the law exact; it only lowers
 *            the acceptance rate).  B_k == 0 reports -1; NaN, negative or +inf
 *            reports -2.
 *   seed, step: Philox key and step counter (advance step between calls).
 *   t_max:   trial budget before the inverse-transform fallback (0 forces the
 *            fallback; 4096 is a good default).
 *   index:   [K] int32 output.  alpha0: NULL or [K] float output, the
 *            fixed-point alpha_0 rounded to float.  trials: NULL or [K]
 *            uint32 output, the accepted trial index + 1, t_max + 1 after the
 *            fallback, 0 for -1/-2/-3.
 * Results are bit-identical to the sequential rule described above.
 */
int arsel_select(arsel_ctx *ctx, const float *alpha, int32_t M, int32_t K, int64_t ld,
                 int layout, const float *bound, uint64_t seed, uint64_t step,
                 uint32_t t_max, uint32_t flags, int32_t *index, float *alpha0,
                 uint32_t *trials, void *stream);

/* Dense-path schedule: at most `tile` instances per workgroup tile (1..64)
 * and `waves` wavefronts per workgroup (4, 8 or 16); tile = waves = 0
 * restores the default (16-instance tiles, 16 wavefronts when the launch has
 * at most one tile per compute unit, else 8).  Results never change. */
int arsel_set_dense_config(arsel_ctx *ctx, int32_t tile, int32_t waves);

/*
 * Trial width of the broadcast kernels (arsel_select with ARSEL_AOS, ld == 0
 * and no bound; arsel_select_proposal with lda == ldq == 0): the vector is
 * staged once per workgroup and each wavefront serves 64 / lanes instances at
 * a time, `lanes` lanes (2 * lanes trials) per instance per round.  lanes is
 * 0 (chosen per launch from the acceptance rate and K) or a power of two in
 * 1..64; ARSEL_ERR_ARG otherwise.  Results never change: trial t of instance
 * k is the same trial for every width and the first accepted one wins.
 */
int arsel_set_trial_lanes(arsel_ctx *ctx, int32_t lanes);

/*
 * Uneven batch: instance k has M_k = offsets[k+1] - offsets[k] reactions at
 * alpha[offsets[k] ..] (AoS).  offsets is a DEVICE array of K+1 int64;
 * host_sizes is NULL or a HOST array of the K sizes.  Instances with M_k up
 * to the schedule's wave_max_m are selected by one wavefront each, staged in
 * LDS.  The larger ones are streamed once for alpha_max and an estimate of
 * alpha_0; those expected to need more than 512 trials are cut into chunks
 * spread over every workgroup, each chunk staged in LDS and tested against
 * all of the instance's trials (so the row is read once more at streaming
 * speed and no candidate costs a DRAM access of its own), and the others run
 * their trials by one wavefront each.  Four launches per call: scan, split,
 * chunks, pick.  With host_sizes the work lists are built on the host,
 * otherwise on the device (three more small launches per call: per-class
 * counts, then placement; the same longest-first order for any K).
 * M_k == 0 reports -1.
 * Results are bit-identical to arsel_select on each instance with instance
 * id k, whatever the schedule, order or split.
 * The context holds this call's work lists and counters: calls on one context
 * must not overlap (issue them on one stream).  A call whose host_sizes and
 * schedule split equal the previous host-sized call's reuses the lists already
 * on the device and makes only the four launches; otherwise the lists are rebuilt and
 * copied through pinned memory.
 * Graph capture: while `stream` captures, host_sizes is ignored and the lists
 * are built on the device inside the graph, so a replay reads no list that a
 * later call leaves in the context.  Buffers the context outgrows are kept
 * until arsel_destroy, so a graph stays valid while its context lives; the
 * schedule is fixed into the graph when it is captured.
 */
int arsel_select_ragged(arsel_ctx *ctx, const float *alpha, const int64_t *offsets,
                        int32_t K, const int64_t *host_sizes, uint64_t seed, uint64_t step,
                        uint32_t t_max, int32_t *index, float *alpha0, uint32_t *trials,
                        void *stream);

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): arsel_select_ragged with
 * the work lists built on the device (as with host_sizes NULL), whose lists,
 * counters, keys and per-instance accumulators live in a static device array
 * of the library instead of the context.  The call makes no allocation of
 * any kind (no hipMalloc, hipFree, pinned host memory or copies) and makes
 * seven launches.  The array holds the state of at most 65536 instances and
 * fixed pools of 2^18 scan items and 2^16 hard chunks (about 12.3 MB); each
 * GPU the library runs on holds its own copy until the process ends.  The
 * chunk plans take the pools' share per instance (up to 32 chunks each), so
 * batches of many instances have longer chunks than arsel_select_ragged.
 * K > 65536: ARSEL_ERR_SIZE; the array's address could not be found when the
 * context was created: ARSEL_ERR_HIP.  Other arguments and results as
 * arsel_select_ragged (bit-identical for any schedule).  Every call on one
 * GPU, from any context, uses that GPU's one array: calls that overlap on a
 * GPU race and must be serialised (one stream, or events between streams).
 * Each call sets every counter it reads and leaves the accumulators zero, so
 * nothing an earlier call left in the array affects it.
 */
int arsel_select_ragged_noalloc(arsel_ctx *ctx, const float *alpha, const int64_t *offsets,
                                int32_t K, uint64_t seed, uint64_t step, uint32_t t_max,
                                int32_t *index, float *alpha0, uint32_t *trials, void *stream);

/*
 * Schedule of arsel_select_ragged (chosen by the autotuner).
 *   wave_max_m:  instances with M <= wave_max_m are run by one wavefront each,
 *                staged in that wave's LDS slice; larger ones are scanned
 *                first and split into easy and hard.
 *   block_waves: wavefronts per workgroup of the pick launch (4, 8 or 16).
 *   lds_max_m:   floats of a hard row staged in LDS at a time by the chunk
 *                launch, also the chunk length (rounded down to a multiple of
 *                4 and clamped to [2048, 16380]; 0 selects 16380).
 *   blocks_per_cu: pick workgroups launched per compute unit (1..8).
 * block_waves * wave_max_m floats (and the hard piece) must fit in one
 * workgroup's LDS (ARSEL_ERR_ARG otherwise).  The schedule never changes
 * results.
 */
typedef struct {
    int32_t wave_max_m;
    int32_t block_waves;
    int32_t lds_max_m;
    int32_t blocks_per_cu;
} arsel_schedule;

int arsel_get_schedule(arsel_ctx *ctx, arsel_schedule *out);
int arsel_set_schedule(arsel_ctx *ctx, const arsel_schedule *s);

/*
 * Acceptance-rejection with an integer proposal Q (the learned proposal):
 * alpha[k*lda + j] (float) and Q[k*ldq + j] (uint32), DEVICE arrays.  Trial t
 * (tag 1 stream) draws V uniform on [0, sum Q) by Lemire's rule on its
 * candidate word, takes the least j with inclusive prefix P_j > V, and accepts
 * when fl64(fl64(u c+) Q_j) < alpha_j, c+ = nextafter(max_j fl64(alpha_j/Q_j)),
 * so the law is alpha_j / alpha_0 for any Q; after t_max rejected trials the
 * same fixed-point inverse transform as arsel_select runs.  index: -4 when
 * Q_j = 0 for some alpha_j > 0, or sum Q >= 2^32 (after the -2 / -1 checks).
 * lda == 0 (ldq == 0) gives every instance the same alpha (Q); otherwise
 * lda, ldq >= M (ARSEL_ERR_LD).  With both 0 the broadcast kernel with packed
 * rounds runs (see arsel_set_trial_lanes).  alpha and the prefix of Q of an
 * instance live in LDS: M up to ~20000 (~10000 in the broadcast kernel, which
 * also keeps Q and a guide table); ARSEL_ERR_SIZE beyond.
 */
int arsel_select_proposal(arsel_ctx *ctx, const float *alpha, const uint32_t *Q, int32_t M,
                          int32_t K, int64_t lda, int64_t ldq, uint64_t seed, uint64_t step,
                          uint32_t t_max, int32_t *index, uint32_t *trials, void *stream);

/*
 * The paper's own scheme (section "A GPU acceptance-rejection algorithm
 * (GPU/AR) for SSA": election and selection steps), for comparison: every
 * reaction j draws u_j = w_j 2^-32 T with T = w * alpha_max (the paper's
 * T_w; w > 0), w_j being word j mod 4 of Philox block j/4 of the tag-3
 * stream (instance k, step); j is eligible when u_j < alpha_j and rated
 * u_j / alpha_j; the eligible reaction with the lowest rating is returned
 * (least index on ties), -5 when none is eligible (the paper's M + 1), -1
 * when every alpha_j is 0, -2 for NaN / negative / +inf.  alpha[k*ld + j]
 * (DEVICE), ld == 0 broadcasts one vector, else ld >= M.  The law of this
 * scheme is NOT alpha_j / alpha_0 (it is biased towards large propensities
 * for small M); bit-identical to the sequential definition.
 */
int arsel_select_paper(arsel_ctx *ctx, const float *alpha, int32_t M, int32_t K, int64_t ld,
                       double w, uint64_t seed, uint64_t step, int32_t *index, void *stream);

/* Mass-action network (DEVICE arrays of M entries): reaction j consumes
 * species r0[j] and, when r1[j] >= 0, r1[j]; it produces p0[j] and, when
 * p1[j] >= 0, p1[j].  Species indices must lie in [0, N). */
typedef struct {
    int32_t N, M;
    const int32_t *r0, *r1, *p0, *p1;
    const float *rate;
} arsel_network;

/* alpha[r*M + j] = rate_j * fl32(h_j(X[r])) with h = x_a, x_a x_b, or
 * x_a (x_a - 1) / 2 (homodimer), computed in int64 and rounded to nearest. */
int arsel_propensities(arsel_ctx *ctx, const arsel_network *net, const int32_t *X, int32_t R,
                       float *alpha, void *stream);

/* The SSA jump chain (the state sequence of the direct method, section "The
 * Stochastic Simulation Algorithm") for R realizations in place on X
 * (int32 [R][N]): step i of realization r selects by uniform AR on the tag-2
 * stream (instance r, step step0 + i) and applies the stoichiometry; an
 * outcome < 0 (nothing can fire) leaves the state.  rec_X (nullable) receives
 * the state before each step i >= rec_from at [(i - rec_from)][r][:]; fired
 * (nullable) the selection of each step at [i][r].  Bit-identical to the
 * sequential definition. */
int arsel_ssa_chain(arsel_ctx *ctx, const arsel_network *net, int32_t *X, int32_t R,
                    uint64_t seed, uint64_t step0, int64_t steps, uint32_t t_max,
                    int64_t rec_from, int32_t *rec_X, int32_t *fired, void *stream);

/* Dependency graph of the full SSA run: deps (DEVICE, [M][ARSEL_SSA_DEP_MAX]
 * int32) lists, for each reaction j, the reactions with a reactant among the
 * species j consumes or produces (the propensities that can change when j
 * fires); ndeps[j] (DEVICE [M]) is their number, or -1 when there are more
 * than ARSEL_SSA_DEP_MAX (then every propensity is recomputed after j). */
#define ARSEL_SSA_DEP_MAX 64
int arsel_ssa_deps(arsel_ctx *ctx, const arsel_network *net, int32_t *deps, int32_t *ndeps,
                   void *stream);

/* Full SSA run, the direct method of section "The Stochastic Simulation
 * Algorithm" with the AR selection: for R realizations (X int32 [R][N] in
 * place, t double [R] in place, DEVICE) and steps i = 0 .. steps-1 (step
 * s = step0 + i), each step selects j with uniform AR on the tag-2 stream
 * (instance r, step s: with period 1 exactly as arsel_ssa_chain), advances t
 * by ln(1/u) / alpha_0 with u = (w + 1/2) 2^-32 from word 0 of Philox block
 * 0xFFFFFFFE of the same stream, applies the stoichiometry and recomputes the
 * propensities of the reactions deps lists for j.
 *
 * The time step's arithmetic is fixed: -ln u by Tang's table-driven method
 * (breakpoints i/128, m in [0.75, 1.5), log1p by its degree-7 series with
 * fused multiply-adds); alpha_0 = fl64(S) 2^-sh with S the sum of
 * floor(alpha_j 2^sh) over the finite positive alpha_j in 128-bit integers,
 * sh = 127 - ceil(log2 M) - E and 2^(E-1) <= alpha_max < 2^E at the scale's
 * last setting: steps with exact envelopes set E, a propensity reaching 2^E
 * drops it, and a step that fires with no E or with S < 2^(95 - ceil(log2 M))
 * takes E from its own alpha_max.  alpha_0 is then the exact sum rounded once
 * to binary64 when the positive propensities lie within 104 - ceil(log2 M)
 * binades of 2^E, and within 2^(2 ceil(log2 M) - 95) of it otherwise.
 *
 * Bound maintenance: the envelope B of the acceptance test (and alpha_0) is
 * exact at the call's first step and at steps with s mod period = 0; between
 * them B is the running maximum of alpha_max since then, kept from the
 * changed propensities, and S is updated by their differences.  Any
 * B >= alpha_max leaves the law alpha_j / alpha_0 of every step; the
 * fallback uses the exact alpha_max.  period 0 or 1: exact at every step (one
 * pass over the M propensities per step); a larger period makes a step read
 * only its candidates and the changed reactions.  Results depend on where
 * calls start, except when they start at multiples of period.
 *
 * Each call first writes a packed copy of the dependency rows ({jj, reactants,
 * rate} per entry) into a buffer of the context (grown on demand, so the first
 * call with a larger M allocates): runs of different networks on one context
 * must not overlap on different streams.
 *
 * An invalid propensity (NaN, negative, +inf) records -2 and no positive one
 * -1; the state and time then stay.  fired (nullable, [steps][R]) and times
 * (nullable, [steps][R], t after each step) are outputs.  States,
 * selections and times are bit-identical to the sequential definition. */
int arsel_ssa_run(arsel_ctx *ctx, const arsel_network *net, const int32_t *deps,
                  const int32_t *ndeps, int32_t *X, int32_t R, uint64_t seed, uint64_t step0,
                  int64_t steps, uint32_t t_max, uint32_t period, double *t, double *times,
                  int32_t *fired, void *stream);

/* The full SSA run selecting with an integer proposal (the learned proposal of
 * the neural-network extension, refreshed lazily by the caller between
 * calls): as arsel_ssa_run, except that each step selects as
 * arsel_select_proposal does (tag-1 stream, instance r, step step0 + i) with
 * Q'_j = max(Q_j, qfloor, 1), Q the DEVICE uint32 row [r][ldq] of realization
 * r (ldq >= M, held fixed for the call), and the envelope C >=
 * max_j fl64(alpha_j / Q'_j), exact at the same steps as B and a running
 * maximum between.  Q' is positive everywhere, so a reaction that becomes
 * active during the call stays covered and each step's law is
 * alpha_j / alpha_0.  qfloor sets the weight of reactions the proposal left
 * out: about sum Q / (8 M) bounds the acceptance rate below by roughly 1/9 of
 * uniform AR's, whatever turns active.  A realization with sum Q' >= 2^32
 * records -4 at every step and does not move.  Q NULL: ARSEL_ERR_NULL;
 * ldq < M: ARSEL_ERR_LD; (N + 2 M) * 4 bytes above one workgroup's LDS:
 * ARSEL_ERR_SIZE. */
int arsel_ssa_run_proposal(arsel_ctx *ctx, const arsel_network *net, const int32_t *deps,
                           const int32_t *ndeps, const uint32_t *Q, int64_t ldq, uint32_t qfloor,
                           int32_t *X, int32_t R, uint64_t seed, uint64_t step0, int64_t steps,
                           uint32_t t_max, uint32_t period, double *t, double *times,
                           int32_t *fired, void *stream);

/* ------------------------------------------------------------------------
 * Learned proposal (BF16 MLP on MFMA, FP32 accumulation).
 *
 * The acceptance-rejection rule stays exact with any proposal Q that covers
 * the support: candidate j is drawn with probability Q_j / sum Q and accepted
 * when u * c+ * Q_j < alpha_j with c+ >= max_j alpha_j / Q_j, so the selection
 * law is alpha_j / alpha_0 whatever the network outputs; a good Q only raises
 * the acceptance rate on skewed propensities.
 * ------------------------------------------------------------------------ */

/* Network description: DEVICE pointers.  f = bf16(log1p(X)) (N inputs,
 * zero-padded to Kp), h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2),
 * z = W3 h2 + b3 (M outputs, rows M..Mp-1 of W3 and b3 are padding).
 * W1: bf16 [H][Kp], W2: bf16 [H][H], W3: bf16 [Mp][H] (row-major, bf16 stored
 * as uint16); b1, b2: float [H]; b3: float [Mp]. */
typedef struct {
    int32_t N, M, H, Kp, Mp;
    const void *W1, *W2, *W3;
    const float *b1, *b2, *b3;
} arsel_mlp;

/* Forward pass for R states X (int32 [R][N] species counts, device) with
 * their propensities alpha (float [R][M], device): q_out (nullable, float
 * [R][M]) = softmax of z over the reactions with alpha_j > 0 (0 elsewhere);
 * Q_out (nullable, uint32 [R][M]) = max(1, floor(q_j 2^(31-L))) on that
 * support, 0 elsewhere, L = ceil(log2 M), so sum Q < 2^32.  Activations live
 * in a context workspace (grown on demand). */
int arsel_mlp_forward(arsel_ctx *ctx, const arsel_mlp *net, const int32_t *X, int32_t R,
                      const float *alpha, float *q_out, uint32_t *Q_out, void *stream);

/* Inference forward path: on != 0 runs arsel_mlp_forward as one fused kernel
 * per block of 32 states (features, the three layers, softmax and
 * quantisation; activations in LDS and registers, no workspace) when
 * H == 256, Kp % 32 == 0, Kp <= 1024, Mp % 16 == 0, Mp <= 1280 and W1, W2,
 * W3 are 16-byte aligned; on == 0 (the default) runs the layer-by-layer
 * kernels.  Both compute the same products and exponentials; q differs only
 * by the order of the softmax row sums (a few ulp). */
int arsel_set_mlp_fused(arsel_ctx *ctx, int32_t on);

/* Training state: the network (its W1, W2, W3 are the BF16 copies refreshed by
 * each step) plus FP32 masters, gradients and Adam moments for the six
 * parameters in the order W1, b1, W2, b2, W3, b3 (shapes as in arsel_mlp).
 * All DEVICE pointers. */
typedef struct {
    arsel_mlp net;
    float *master[6];
    float *grad[6];
    float *m[6];
    float *v[6];
    float beta1, beta2, eps;
} arsel_mlp_train;

/* One Adam step (t = 1, 2, ...) on a minibatch of B (state, propensity)
 * pairs: loss = mean over rows of the cross-entropy -sum_j p_j log q_j with
 * p = alpha / alpha_0 on the support; gradients by the backward GEMMs on
 * MFMA; *loss (device float) receives the minibatch loss. */
int arsel_mlp_train_step(arsel_ctx *ctx, const arsel_mlp_train *tr, const int32_t *X,
                         const float *alpha, int32_t B, float lr, int32_t t, float *loss,
                         void *stream);

/* Refresh the BF16 copies (net.W1, W2, W3) from the FP32 masters
 * (nearest-even rounding); used after initialising or loading masters. */
int arsel_mlp_sync_bf16(arsel_ctx *ctx, const arsel_mlp_train *tr, void *stream);

/* C = A . B^T-style product on MFMA: C[m][n] = sum_k A(m,k) B(n,k), BF16 A and
 * B (device), FP32 C [M][ldc]; A(m,k) = A[m*lda+k] if a_kcontig else
 * A[k*lda+m]; B(n,k) = B[n*ldb+k] if b_kcontig else B[k*ldb+n]; optional
 * bias[n] and ReLU.  The building block of the MLP kernels. */
int arsel_gemm_bf16(arsel_ctx *ctx, const void *A, int64_t lda, int32_t a_kcontig, const void *B,
                    int64_t ldb, int32_t b_kcontig, int32_t M, int32_t N, int32_t K,
                    const float *bias, int32_t relu, float *C, int64_t ldc, void *stream);

/* ------------------------------------------------------------------------
 * Measurement utility (not part of the method).
 *
 * Read bandwidth the device reaches on a rows x cols float matrix (DEVICE,
 * row stride ld floats, 16-byte aligned, ld % 4 == 0) read once with the
 * selection kernels' own 16-byte non-temporal loads, all of a workgroup's
 * loads issued before any is consumed; timing it gives the achievable ceiling
 * beside the data-sheet peak.
 *   tile == 0: the matrix as one contiguous span (cols == ld), 4096 float4
 *              per workgroup of 1024 threads;
 *   tile in {4, 8, 16, 32, 64}, cols % tile == 0: the dense SoA pattern of
 *              arsel_select: workgroup b reads `tile` consecutive columns of
 *              every row (the XCD-aware tile order of the dense kernel).
 * *grid_out receives the number of workgroups; sink (DEVICE, sink_len >= that
 * number of uint32) receives each workgroup's maximum of the bits it read, so
 * that no load can be dropped.  sink_len too small or more than 2^31 - 1
 * workgroups: ARSEL_ERR_SIZE (nothing launched); a bad tile: ARSEL_ERR_ARG.
 */
int arsel_probe_read(arsel_ctx *ctx, const float *p, int32_t rows, int32_t cols, int64_t ld,
                     int32_t tile, uint32_t *sink, int64_t sink_len, int64_t *grid_out,
                     void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ARSEL_H */
