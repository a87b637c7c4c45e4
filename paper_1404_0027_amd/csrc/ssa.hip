// Mass-action propensities, the SSA jump chain (training data for the
// learned proposal) and the full SSA run (direct method with the time step).
//
// Reaction j of the network consumes species r0[j] (and r1[j] when >= 0) and
// produces p0[j] (and p1[j] when >= 0).  Its propensity is
// alpha_j = rate_j * fl32(h) with the combinatorial count h (int64): x_a for
// one reactant, x_a x_b for two distinct ones, x_a (x_a - 1) / 2 for a
// homodimer; fl32 rounds to nearest even.  The jump chain is the sequence of
// states of the direct method (section "The Stochastic Simulation
// Algorithm": select j, then X <- X + v_j); the holding times do not change
// it, so they are not drawn.  Step i of realization r selects with uniform
// acceptance-rejection on the tag-2 stream (instance r, step step0 + i).
#include "launch.hpp"
#include "proposal_core.hpp"
#include "select_core.hpp"

namespace arsel {

__device__ __forceinline__ float mass_action(const int32_t *x, int32_t a, int32_t b, float rate)
{
    int64_t h;
    if (b < 0)
        h = x[a];
    else if (b == a)
        h = (int64_t)x[a] * (x[a] - 1) / 2;
    else
        h = (int64_t)x[a] * x[b];
    // nearest-even conversion of a non-negative count (h >= 0 for counts >= 0):
    // the hardware conversion below 2^32, the exact 64-bit one above
    const float fh = h <= 0 ? 0.0f
                     : h < (1ll << 32) ? (float)(uint32_t)h
                                       : fixed_to_float((uint64_t)h, 0);
    return rate * fh;
}

struct NetArgs {
    const int32_t *r0, *r1, *p0, *p1;
    const float *rate;
    int32_t N, M;
};

__global__ void k_propensities(NetArgs n, const int32_t *X, int32_t R, float *alpha)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)R * n.M) return;
    const int64_t r = idx / n.M;
    const int j = (int)(idx - r * n.M);
    alpha[idx] = mass_action(X + r * n.N, n.r0[j], n.r1[j], n.rate[j]);
}

struct ChainArgs {
    NetArgs net;
    int32_t *X;          // [R][N], updated in place
    int32_t R;
    uint64_t seed, step0;
    int64_t steps;
    uint32_t t_max;
    int64_t rec_from;
    int32_t *rec_X;      // [(steps - rec_from)][R][N] or null
    int32_t *fired;      // [steps][R] or null
};

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront per realization: state and propensities in that wave's LDS.
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_ssa_chain(ChainArgs c)
{
    extern __shared__ int32_t lds_i[];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int r = blockIdx.x * NW + wave;
    if (r >= c.R) return;
    const int N = c.net.N, M = c.net.M;
    int32_t *x = lds_i + (size_t)wave * (N + M);
    float *a = reinterpret_cast<float *>(x + N);
    int32_t *gx = c.X + (int64_t)r * N;
    for (int i = lane; i < N; i += kWave) x[i] = gx[i];
    wave_sync_lds();
    for (int64_t i = 0; i < c.steps; ++i) {
        if (c.rec_X && i >= c.rec_from) {
            int32_t *dst = c.rec_X + ((i - c.rec_from) * c.R + r) * (int64_t)N;
            for (int s = lane; s < N; s += kWave) dst[s] = x[s];
        }
        for (int j = lane; j < M; j += kWave)
            a[j] = mass_action(x, c.net.r0[j], c.net.r1[j], c.net.rate[j]);
        wave_sync_lds();
        const Stream st = make_stream(c.seed, c.step0 + (uint64_t)i, (uint32_t)r, kTagSSA);
        const Outcome o = wave_select(ContigAcc{a}, (uint32_t)M, nullptr, 0u, st, c.t_max, false);
        const int32_t j = (int32_t)uniform_u32((uint32_t)o.index);
        if (c.fired && lane == 0) c.fired[i * c.R + r] = j;
        if (j >= 0 && lane == 0) {
            x[c.net.r0[j]] -= 1;
            if (c.net.r1[j] >= 0) x[c.net.r1[j]] -= 1;
            x[c.net.p0[j]] += 1;
            if (c.net.p1[j] >= 0) x[c.net.p1[j]] += 1;
        }
        wave_sync_lds();
    }
    for (int i = lane; i < N; i += kWave) gx[i] = x[i];
}

// Reactions whose propensity can change when reaction j fires: those with a
// reactant among the species j consumes or produces.  deps[j][0 .. ndeps[j])
// lists them; ndeps[j] = -1 when there are more than kDepMax (the run then
// recomputes every propensity after j).
constexpr int kDepMax = ARSEL_SSA_DEP_MAX;

__global__ void k_ssa_deps(NetArgs n, int32_t *deps, int32_t *ndeps)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n.M) return;
    const int s0 = n.r0[j], s1 = n.r1[j], s2 = n.p0[j], s3 = n.p1[j];
    int cnt = 0;
    for (int i = 0; i < n.M; ++i) {
        const int a = n.r0[i], b = n.r1[i];
        const bool hit = a == s0 || a == s1 || a == s2 || a == s3 ||
                         (b >= 0 && (b == s0 || b == s1 || b == s2 || b == s3));
        if (hit) {
            if (cnt < kDepMax) deps[(int64_t)j * kDepMax + cnt] = i;
            ++cnt;
        }
    }
    ndeps[j] = cnt <= kDepMax ? cnt : -1;
}

constexpr uint32_t kTauBlock = 0xFFFFFFFEu;

// -ln(u) for u = (w + 1/2) 2^-32, table-driven (P. T. P. Tang, "Table-driven
// implementation of the logarithm function in IEEE floating-point
// arithmetic", ACM TOMS 16, 1990): u = v 2^-33 with v = 2w + 1 exact, written
// as m 2^e with m in [0.75, 1.5); c = i / 128 is the grid point nearest m
// (so m - c is exact and r = (m - c) / c has |r| <= 2^-8 / 0.75), and
// ln u = e ln 2 + ln c + log1p(r) with log1p by its Taylor series to degree 7
// (the first omitted term is below 2^-56 relative).  Near u = 1, e = 0 and
// c = 1 (ln c = 0), so the result keeps its relative accuracy there.  tab
// holds {ln c_i, 1 / c_i} for i = 96 .. 192.
__device__ __forceinline__ double neg_ln_u(uint32_t w, const double *tab)
{
    const uint64_t v = 2ull * w + 1ull;
    const int n = 64 - __clzll((long long)v);             // 2^(n-1) <= v < 2^n
    double m = ldexp((double)v, 1 - n);                    // [1, 2)
    int e = n - 34;
    if (m >= 1.5) {
        m *= 0.5;
        e += 1;
    }
    const int i = (int)rint(m * 128.0);
    const double lnc = tab[2 * (i - kLnTabLo)], inv = tab[2 * (i - kLnTabLo) + 1];
    const double r = (m - (double)i * 0x1p-7) * inv;
    double p = 1.0 / 7.0;
    p = fma(p, r, -1.0 / 6.0);
    p = fma(p, r, 1.0 / 5.0);
    p = fma(p, r, -1.0 / 4.0);
    p = fma(p, r, 1.0 / 3.0);
    p = fma(p, r, -1.0 / 2.0);
    p = fma(p, r, 1.0);
    const double l1p = p * r;
    return -((fma((double)e, 0.69314718055994530942, lnc)) + l1p);
}

// ---- alpha_0 of the time step in 128-bit fixed point ----
//
// With a scale exponent E (2^(E-1) <= a maximum of the propensities < 2^E)
// and sh = 127 - L - E, L = ceil(log2 M), the propensity with bits b weighs
// F(b) = floor(v 2^sh) < 2^(127-L) when v is finite and positive, 0
// otherwise; S = sum_j F(b_j) < 2^127 is exact, and alpha_0 = fl64(S) 2^-sh
// is rounded once.  Every v >= 2^(E-103+L) is a whole multiple of 2^-sh, so
// when the positive propensities lie within 104 - L binades of 2^E alpha_0
// is their exact sum rounded once, whatever their order.  The run keeps S
// from the changed propensities' differences (mod 2^128) and rebuilds it
// when E changes.  E is set at the steps with exact envelopes to that of
// alpha_max, stays while every valid propensity is below 2^E, and is
// dropped when one reaches it; a step that fires with no E, or with
// S < 2^(95-L) (alpha_0 fell 32 binades below 2^E), takes E from its own
// alpha_max, so the dropped parts stay below 2^(2L-95) of alpha_0.
struct U128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ U128 add128(U128 a, U128 b)
{
    U128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (uint64_t)(r.lo < a.lo);
    return r;
}

__device__ __forceinline__ U128 sub128(U128 a, U128 b)
{
    U128 r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (uint64_t)(a.lo < b.lo);
    return r;
}

constexpr int kNoScale = -100000;

// F(b) at the shift sh: v = m 2^(max(e,1) - 150) with m the 24-bit
// significand, so F = m 2^k with k = max(e,1) - 150 + sh, k <= 103 for
// v < 2^E.  The low word is m << k (k in 0..63) or m >> -k (k < 0); the high
// word holds m >> (64 - k) for k in 41..63 and m << (k - 64) for k >= 64.
// Shift amounts are masked to 0..63; values at or above 2^E (which drop the
// scale) give some value that is never used.
__device__ __forceinline__ U128 wide_weight(uint32_t b, int sh)
{
    const uint32_t e = b >> 23;
    const uint64_t m = b < 0x7F800000u ? (uint64_t)((b & 0x7FFFFFu) | (e ? 0x800000u : 0u)) : 0ull;
    const int k = (int)max(e, 1u) - 150 + sh;
    const uint64_t up = m << (k & 63);
    const uint64_t dn = m >> (min(-k, 63) & 63);
    const uint64_t sp = m >> ((64 - k) & 63);
    U128 r;
    r.lo = k >= 64 ? 0ull : (k >= 0 ? up : dn);
    r.hi = k >= 64 ? up : (k > 40 ? sp : 0ull);
    return r;
}

// F(nv) - F(old) mod 2^128, invalid values counting as 0.  When the
// smaller nonzero exponent puts both on the grid (k >= 0) and the two lie
// within 38 binades, their significands aligned to that exponent differ by
// an exact int64 delta and the difference is delta 2^k; otherwise the two
// weights are taken apart.
__device__ __forceinline__ U128 wide_delta(float old, float nv, int sh)
{
    const uint32_t bo = __float_as_uint(old), bn = __float_as_uint(nv);
    const uint32_t co = bo < 0x7F800000u ? bo : 0u, cn = bn < 0x7F800000u ? bn : 0u;
    const uint32_t eo = co >> 23, en = cn >> 23;
    const uint64_t mo = (co & 0x7FFFFFu) | (eo ? 0x800000u : 0u);
    const uint64_t mn = (cn & 0x7FFFFFu) | (en ? 0x800000u : 0u);
    const int xo = (int)max(eo, 1u), xn = (int)max(en, 1u);
    const int xb = min(co ? xo : 255, cn ? xn : 255);   // 255: both zero, delta 0
    const int go = xo - xb, gn = xn - xb;         // a zero value may give < 0: its m is 0
    const int k = xb - 150 + sh;
    U128 r;
    if (k >= 0 && max(go, gn) <= 38) {
        const int64_t dl = (int64_t)(mn << (gn & 63)) - (int64_t)(mo << (go & 63));
        const uint64_t sl = (uint64_t)dl << (k & 63);
        const uint64_t sr = (uint64_t)(dl >> ((64 - k) & 63));
        r.lo = k < 64 ? sl : 0ull;
        r.hi = k >= 64 ? sl : (k == 0 ? (uint64_t)(dl >> 63) : sr);
    } else {
        r = sub128(wide_weight(cn, sh), wide_weight(co, sh));
    }
    return r;
}

// Bits of the float 2^E (E in -148..128; 2^128 gives the bits of +inf, which
// no finite value reaches).
__device__ __forceinline__ uint32_t pow2_bits(int E)
{
    return E >= -126 ? (uint32_t)(E + 127) << 23 : 1u << (E + 149);
}

// fl64(S) 2^-sh, rounded to nearest even once: for S >= 2^64 the top 64
// bits are converted with the bits below them folded into the last bit
// (they lie below the rounding position), then scaled back.  S < 2^127.
__device__ __forceinline__ double wide_to_f64(U128 s, int sh)
{
    const int n = s.hi ? 64 - __clzll((long long)s.hi) : 0;     // 0..63
    const uint64_t top = n ? (s.hi << ((64 - n) & 63)) | (s.lo >> n) |
                                 (uint64_t)((s.lo << ((64 - n) & 63)) != 0)
                           : s.lo;
    return ldexp((double)top, n - sh);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ U128 dpp_add128(U128 x)
{
    U128 y;
    y.lo = dpp_u64<CTRL, ROW_MASK>(x.lo);
    y.hi = dpp_u64<CTRL, ROW_MASK>(x.hi);
    return add128(x, y);
}

__device__ __forceinline__ U128 readlane128(U128 x, int l)
{
    U128 r;
    r.lo = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x.lo, l) |
           ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x.lo >> 32), l) << 32);
    r.hi = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x.hi, l) |
           ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x.hi >> 32), l) << 32);
    return r;
}

__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    return __longlong_as_double((long long)(
        (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l) |
        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l) << 32)));
}

// Sums mod 2^128 over the wavefront, over lanes 0..15, and over each 32-lane
// half (the DPP patterns of the binary64 sums); every lane returns its sum.
__device__ __forceinline__ U128 wave_sum_u128(U128 x)
{
    x = dpp_add128<0x111>(x);
    x = dpp_add128<0x112>(x);
    x = dpp_add128<0x114>(x);
    x = dpp_add128<0x118>(x);
    x = dpp_add128<0x142, 0xA>(x);
    x = dpp_add128<0x143, 0xC>(x);
    return readlane128(x, 63);
}

// Sum of lanes 0..15 (row 0); every lane returns it.
__device__ __forceinline__ U128 row0_sum_u128(U128 x)
{
    x = dpp_add128<0x111>(x);
    x = dpp_add128<0x112>(x);
    x = dpp_add128<0x114>(x);
    x = dpp_add128<0x118>(x);
    return readlane128(x, 15);
}

struct RunArgs {
    NetArgs net;
    const int32_t *deps, *ndeps;
    int32_t *X;          // [R][N], updated in place
    int32_t R;
    uint64_t seed, step0;
    int64_t steps;
    uint32_t t_max;
    double *t;           // [R], advanced in place
    double *times;       // [steps][R] or null
    int32_t *fired;      // [steps][R] or null
    const uint32_t *Q;   // [R][ldq] integer proposal (proposal run only)
    int64_t ldq;
    uint32_t qfloor;     // Q'_j = max(Q_j, qfloor, 1)
    uint32_t period;     // exact envelopes every period steps (0 or 1: every step)
    const int4 *tab;     // [M][kDepMax] {jj, r0[jj], r1[jj], rate[jj] bits} of deps
    const double *ln_tab;
};

// Uniform AR of one step on alpha in LDS with the envelope env: the rounds of
// the sequential rule, trial t in Philox block t / 2 of the tag-2 stream
// (words 0, 1 for even t, 2, 3 for odd t).  The first round's lane 63 draws
// block 0xFFFFFFFE instead (the time step's), so that round covers blocks
// 0..62 and round k >= 1 blocks 63 + 64 (k - 1) .. + 63; tau_w is word 0 of
// block 0xFFFFFFFE.  After t_max trials the exact fallback runs.
__device__ __forceinline__ Outcome ssa_uniform_rounds(const float *a, uint32_t M, float env,
                                                      bool scanned, const Stream &st,
                                                      uint32_t t_max, uint32_t &tau_w)
{
    const int lane = lane_id();
    const uint32_t thresh = lemire_threshold(M);
    const double envd = (double)env;
    uint64_t key = kNoAccept;
    uint32_t first = 0;      // first block of the round
    bool round0 = true;
    do {
        const bool taul = round0 && lane == kWave - 1;
        const uint32_t b = taul ? kTauBlock : first + (uint32_t)lane;
        const Words w = st.block(b);
        if (round0) tau_w = readlane_u32(w.w0, kWave - 1);
        const uint64_t ta = 2 * (uint64_t)b;
        uint32_t ja = 0, jb = 0;
        const bool oka = !taul && lemire(w.w0, M, thresh, ja) && ta < t_max;
        const bool okb = !taul && lemire(w.w2, M, thresh, jb) && ta + 1 < t_max;
        const bool acca = oka && grid_u(w.w1) * envd < (double)a[ja];
        const bool accb = okb && grid_u(w.w3) * envd < (double)a[jb];
        const uint64_t ma = __ballot(acca), mb = __ballot(accb);
        if (ma | mb) {
            const int la = first_lane(ma), lb = first_lane(mb);
            key = la <= lb ? ((2 * (uint64_t)(first + la)) << 32) | readlane_u32(ja, la)
                           : ((2 * (uint64_t)(first + lb) + 1) << 32) | readlane_u32(jb, lb);
        }
        first += round0 ? kWave - 1 : kWave;
        round0 = false;
    } while (key == kNoAccept && 2 * (uint64_t)first < t_max);
    if (key != kNoAccept) {
        Outcome o;
        o.index = (int32_t)(uint32_t)key;
        o.trials = (uint32_t)(key >> 32) + 1;
        o.alpha0 = 0.0f;
        return o;
    }
    return wave_fallback(ContigAcc{a}, M, scanned, env, st, t_max, 0.0f);
}

// Row j of the packed dependency table: entry l < ndeps[j] holds reaction
// jj = deps[j][l] with its reactants and rate, so the run's update reads one
// 16-byte entry per affected reaction; other entries hold {-1, 0, -1, 0}.
__global__ void k_ssa_pack(NetArgs n, const int32_t *deps, const int32_t *ndeps, int4 *tab)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n.M * kDepMax) return;
    const int j = (int)(i / kDepMax), l = (int)(i % kDepMax);
    int4 e = make_int4(-1, 0, -1, 0);
    if (l < ndeps[j]) {
        const int jj = deps[i];
        e = make_int4(jj, n.r0[jj], n.r1[jj], __float_as_int(n.rate[jj]));
    }
    tab[i] = e;
}

// Valid propensity: non-negative (-0.0 included) and finite.
__device__ __forceinline__ bool valid_prop(float v)
{
    return v >= 0.0f && v != __builtin_inff();
}

// Sum over the wavefront of two signed counts (|sum| < 2^31 each).
__device__ __forceinline__ void wave_sum_pair(int32_t &a, int32_t &b)
{
    a = (int32_t)wave_sum_u32((uint32_t)a);
    b = (int32_t)wave_sum_u32((uint32_t)b);
}

// One wavefront per realization, counts and propensities in its LDS.  Each
// step selects the next reaction with the envelope of the step, advances the
// time by tau = ln(1/u) / alpha_0 (u from Philox block 0xFFFFFFFE of the
// tag-2 stream), applies the stoichiometry and recomputes the propensities of
// the reactions the fired one affects (the dependency graph).
//
// Bound maintenance with period p: at the call's first step and at steps
// s with s mod p = 0 one pass over the propensities takes the exact
// alpha_max (the envelope B), the numbers of positive and of invalid
// propensities and, with a proposal, the exact c; between those steps the
// update of the affected reactions keeps the counts and the running maxima
// B and C, so a step reads only its candidates and the changed reactions.
// alpha_0 of the time step is the 128-bit fixed-point sum S (above), kept
// from the changed reactions' differences at every period.  B >= alpha_max
// and C >= max_j alpha_j / Q'_j keep each step's law alpha_j / alpha_0; the
// fallback still uses the exact alpha_max.  p = 1 takes the pass at every
// step.
//
// PROP = false selects with uniform AR on the tag-2 stream (the jump
// chain's); PROP = true with the integer proposal Q'_j = max(Q_j, qfloor, 1)
// of the realization (its inclusive prefix kept in LDS for the whole call)
// on the tag-1 stream.  An invalid propensity gives -2 and no positive one
// -1 (both permanent: nothing fires), sum Q' >= 2^32 gives -4.
template <int NW, bool PROP>
__global__ __launch_bounds__(NW * 64, PROP ? 1 : 6) void k_ssa_run(RunArgs c)
{
    static_assert(kDepMax == kWave, "one dependency row per wavefront load");
    extern __shared__ int32_t lds_i[];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int r = blockIdx.x * NW + wave;
    if (r >= c.R) return;
    const int N = c.net.N, M = c.net.M;
    int32_t *x = lds_i + (size_t)wave * (N + (PROP ? 2 : 1) * M);
    float *a = reinterpret_cast<float *>(x + N);
    uint32_t *sp = reinterpret_cast<uint32_t *>(a + M);   // prefix of Q' (PROP)
    int32_t *gx = c.X + (int64_t)r * N;
    for (int i = lane; i < N; i += kWave) x[i] = gx[i];
    uint64_t sumq = 0;
    if (PROP) {
        const uint32_t *gq = c.Q + (int64_t)r * c.ldq;
        const uint32_t lo = max(c.qfloor, 1u);
        for (int j = lane; j < M; j += kWave) {
            const uint32_t q = max(gq[j], lo);
            sp[j] = q;
            sumq += q;
        }
        sumq = wave_sum_u64(sumq);
    }
    wave_sync_lds();
    if (PROP) wave_prefix_u32([&](uint32_t j) { return sp[j]; }, sp, (uint32_t)M);
    for (int j = lane; j < M; j += kWave) a[j] = mass_action(x, c.net.r0[j], c.net.r1[j], c.net.rate[j]);
    wave_sync_lds();
    auto qat = [&](uint32_t jj) { return sp[jj] - (jj ? sp[jj - 1] : 0u); };
    const uint64_t period = max(c.period, 1u);
    const bool maintain = period > 1;   // with period 1 the envelopes are not kept across steps
    const int L = ceil_log2_u32((uint32_t)M);
    double t = c.t[r];
    // the time steps of a batch of up to 64 steps: lane k holds step b0 + k's
    // Philox word and alpha_0; the logarithms and quotients are taken in
    // parallel at the batch's end and added to t in step order
    uint32_t bw = 0;
    double ba = 1.0;
    uint64_t fmask = 0;  // steps of the batch that fired
    int64_t b0 = 0;
    auto flush = [&](int64_t iend) {
        const int n = (int)(iend - b0);
        const double tau = ((fmask >> lane) & 1) ? neg_ln_u(bw, c.ln_tab) / ba : 0.0;
        double tk = t;
        for (int k = 0; k < n; ++k) {
            if ((fmask >> k) & 1) t += readlane_f64(tau, k);
            tk = lane == k ? t : tk;
        }
        if (c.times && lane < n) c.times[(b0 + lane) * c.R + r] = tk;
        fmask = 0;
        b0 = iend;
    };
    U128 S{0, 0};        // sum of F at the scale Es (when have)
    int Es = kNoScale;
    bool have = false;
    float B = 0.0f;      // envelope >= alpha_max (uniform)
    double C = 0.0;      // envelope >= max_j alpha_j / Q'_j (proposal)
    int32_t npos = 0, nbad = 0;
    for (int64_t i = 0; i < c.steps; ++i) {
        const uint64_t s = c.step0 + (uint64_t)i;
        const bool exact = i == 0 || s % period == 0;
        if (exact) {
            uint32_t mb = 0;
            float rmax = 0.0f;
            if (maintain) {
                npos = 0;
                nbad = 0;
                for (int j = lane; j < M; j += kWave) {
                    const float v = a[j];
                    mb = max(mb, __float_as_uint(v) & 0x7FFFFFFFu);   // alpha_max while all are valid
                    npos += v > 0.0f;
                    nbad += !valid_prop(v);
                    if (PROP && v > 0.0f) rmax = fmaxf(rmax, ratio_estimate(v, qat((uint32_t)j)));
                }
                B = __uint_as_float(wave_max_u32(mb));
                wave_sum_pair(npos, nbad);
            } else {
                // the raw bit maximum certifies validity and is alpha_max below
                // 0x7F800000; otherwise an exact scan decides
                for (int j = lane; j < M; j += kWave) {
                    const float v = a[j];
                    mb = max(mb, __float_as_uint(v));
                    if (PROP && v > 0.0f) rmax = fmaxf(rmax, ratio_estimate(v, qat((uint32_t)j)));
                }
                mb = wave_max_u32(mb);
                bool bad = false;
                if (mb < 0x7F800000u)
                    B = __uint_as_float(mb);
                else
                    wave_scan(ContigAcc{a}, (uint32_t)M, B, bad);
                nbad = bad ? 1 : 0;
                npos = B > 0.0f ? 1 : 0;
            }
            if (nbad == 0 && npos > 0) {
                const int e = exponent_above(B);      // B is alpha_max here
                if (e != Es) {
                    Es = e;
                    have = false;
                }
            } else {
                Es = kNoScale;
                have = false;
            }
            if (PROP && nbad == 0 && npos > 0 && sumq < (1ull << 32))
                C = wave_proposal_c_band(a, (uint32_t)M, qat, wave_max_f32_nonneg(rmax));
        }
        Outcome o;
        uint32_t tau_w = 0;     // word 0 of the time step's Philox block
        if (nbad != 0) {
            o.index = -2;
        } else if (npos == 0) {
            o.index = -1;
        } else if (PROP) {
            if (sumq >= (1ull << 32)) {
                o.index = -4;
            } else {
                const double cplus = __longlong_as_double(__double_as_longlong(C) + 1);
                const Stream sq = make_stream(c.seed, s, (uint32_t)r, kTagProposal);
                o = wave_proposal_rounds(a, sp, (uint32_t)M, (uint32_t)sumq, cplus,
                                         exact ? B : -1.0f, sq, c.t_max);
                tau_w = make_stream(c.seed, s, (uint32_t)r, kTagSSA).block(kTauBlock).w0;
            }
        } else {
            // at a non-exact step the fallback takes the exact maximum itself
            o = ssa_uniform_rounds(a, (uint32_t)M, B, exact,
                                   make_stream(c.seed, s, (uint32_t)r, kTagSSA), c.t_max, tau_w);
        }
        const int32_t j = (int32_t)uniform_u32((uint32_t)o.index);
        if (c.fired && lane == 0) c.fired[i * c.R + r] = j;
        if (j >= 0) {
            // reaction j's stoichiometry, dependency count and whole dependency
            // row (in bounds: the table is [M][kDepMax]) issued together
            const int32_t nd = c.ndeps[j];
            const int4 dl = c.tab[(int64_t)j * kDepMax + lane];
            const int32_t jr0 = c.net.r0[j], jr1 = c.net.r1[j], jp0 = c.net.p0[j], jp1 = c.net.p1[j];
            if (have && S.hi < (1ull << (31 - L))) {       // alpha_0 < 2^(Es-32)
                Es = kNoScale;
                have = false;
            }
            if (!have) {
                if (Es == kNoScale) {
                    uint32_t mb = 0;
                    for (int jj = lane; jj < M; jj += kWave)
                        mb = max(mb, __float_as_uint(a[jj]) & 0x7FFFFFFFu);
                    Es = exponent_above(__uint_as_float(wave_max_u32(mb)));
                }
                const int sh = 127 - L - Es;
                U128 acc{0, 0};
                for (int jj = lane; jj < M; jj += kWave)
                    acc = add128(acc, wide_weight(__float_as_uint(a[jj]), sh));
                S = wave_sum_u128(acc);
                have = true;
            }
            const int sh = 127 - L - Es;
            {
                const int slot = (int)(i - b0);
                const double a0 = wide_to_f64(S, sh);
                if (lane == slot) {
                    bw = uniform_u32(tau_w);
                    ba = a0;
                }
                fmask |= 1ull << slot;
            }
            if (lane == 0) {
                x[jr0] -= 1;
                if (jr1 >= 0) x[jr1] -= 1;
                x[jp0] += 1;
                if (jp1 >= 0) x[jp1] += 1;
            }
            wave_sync_lds();
            // S from the changed reactions' differences; a valid new value at
            // or above 2^Es drops the scale
            const uint32_t sthr = pow2_bits(Es);
            U128 d{0, 0};
            bool up = false;
            auto track = [&](float old, float nv) {
                d = add128(d, wide_delta(old, nv, sh));
                up |= __float_as_uint(nv) < 0x7F800000u && __float_as_uint(nv) >= sthr;
            };
            if (maintain) {
                // count changes from ballots (wave-uniform), the envelope only
                // when a new value exceeds it
                double cm = 0.0;
                uint32_t bm = 0;
                auto update = [&](bool on, int jj, int32_t ra, int32_t rb, float k) {
                    float old = 0.0f, nv = 0.0f;
                    if (on) {
                        old = a[jj];
                        nv = mass_action(x, ra, rb, k);
                        a[jj] = nv;
                        track(old, nv);
                        if (valid_prop(nv)) {
                            if (!PROP) bm = max(bm, __float_as_uint(nv) & 0x7FFFFFFFu);
                            if (PROP && nv > 0.0f)
                                cm = fmax(cm, (double)nv / (double)qat((uint32_t)jj));
                        }
                    }
                    npos += __popcll(__ballot(on && nv > 0.0f)) - __popcll(__ballot(on && old > 0.0f));
                    nbad += __popcll(__ballot(on && !valid_prop(nv))) -
                            __popcll(__ballot(on && !valid_prop(old)));
                };
                if (nd < 0) {
                    for (int base = 0; base < M; base += kWave) {
                        const int jj = base + lane;
                        const bool on = jj < M;
                        update(on, jj, on ? c.net.r0[jj] : 0, on ? c.net.r1[jj] : -1,
                               on ? c.net.rate[jj] : 0.0f);
                    }
                } else {
                    update(lane < nd, dl.x, dl.y, dl.z, __int_as_float(dl.w));
                }
                if (PROP) {
                    if (__ballot(cm > C)) C = fmax(C, wave_max_f64_nonneg(cm));
                } else {
                    if (__ballot(bm > __float_as_uint(B))) B = fmaxf(B, __uint_as_float(wave_max_u32(bm)));
                }
            } else {
                auto update = [&](int jj, int32_t ra, int32_t rb, float k) {
                    const float old = a[jj], nv = mass_action(x, ra, rb, k);
                    a[jj] = nv;
                    track(old, nv);
                };
                if (nd < 0) {
                    for (int jj = lane; jj < M; jj += kWave)
                        update(jj, c.net.r0[jj], c.net.r1[jj], c.net.rate[jj]);
                } else if (lane < nd) {
                    update(dl.x, dl.y, dl.z, __int_as_float(dl.w));
                }
            }
            S = add128(S, (nd >= 0 && nd <= 16) ? row0_sum_u128(d) : wave_sum_u128(d));
            if (__ballot(up)) {
                Es = kNoScale;
                have = false;
            }
            wave_sync_lds();
        }
        if (i + 1 - b0 == kWave) flush(i + 1);
    }
    if (b0 < c.steps) flush(c.steps);
    for (int i = lane; i < N; i += kWave) gx[i] = x[i];
    if (lane == 0) c.t[r] = t;
}

// ---- two realizations per wavefront (uniform AR) ----
//
// Half h of a wavefront (lanes 32h .. 32h + 31) runs realization 2w + h with
// the steps of k_ssa_run<NW, false>, each half doing what the whole wave
// does there; the results are identical (same trials, same fallback, same
// envelopes).  One wavefront's instruction stream then serves two
// realizations, which pays because that kernel's step is issue-bound.
// Rounds cover 32 Philox blocks per half (the first round 31 trial blocks
// and the time step's block in lane 31 of the half).

// Sums / maxima over each half by DPP row shifts and one row broadcast: half
// 0's total ends in lane 31, half 1's in lane 63; every lane returns its
// half's.
__device__ __forceinline__ uint32_t half_pick(uint32_t v0, uint32_t v1)
{
    return (lane_id() & 32) ? v1 : v0;
}

__device__ __forceinline__ uint32_t half_sum_u32(uint32_t x)
{
    x += dpp_u32<0x111>(x);
    x += dpp_u32<0x112>(x);
    x += dpp_u32<0x114>(x);
    x += dpp_u32<0x118>(x);
    x += dpp_u32<0x142, 0xA>(x);     // row_bcast:15 into rows 1 and 3
    return half_pick((uint32_t)__builtin_amdgcn_readlane((int)x, 31),
                     (uint32_t)__builtin_amdgcn_readlane((int)x, 63));
}

__device__ __forceinline__ uint32_t half_max_u32(uint32_t x)
{
    x = max(x, dpp_u32<0x111>(x));
    x = max(x, dpp_u32<0x112>(x));
    x = max(x, dpp_u32<0x114>(x));
    x = max(x, dpp_u32<0x118>(x));
    x = max(x, dpp_u32<0x142, 0xA>(x));
    return half_pick((uint32_t)__builtin_amdgcn_readlane((int)x, 31),
                     (uint32_t)__builtin_amdgcn_readlane((int)x, 63));
}

__device__ __forceinline__ U128 half_sum_u128(U128 x)
{
    x = dpp_add128<0x111>(x);
    x = dpp_add128<0x112>(x);
    x = dpp_add128<0x114>(x);
    x = dpp_add128<0x118>(x);
    x = dpp_add128<0x142, 0xA>(x);
    const U128 s0 = readlane128(x, 31), s1 = readlane128(x, 63);
    return (lane_id() & 32) ? s1 : s0;
}

// 64-bit shuffles within the 32-lane half (the fallback's rare path).
__device__ __forceinline__ uint64_t half_shfl_xor_u64(uint64_t x, int off)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, off, 32);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), off, 32);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t half_shfl_up_u64(uint64_t x, int d)
{
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, 32);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, 32);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// The exact fixed-point inverse transform of one half's instance (valid
// propensities, at least one positive): the arithmetic of wave_fallback over
// 32 lanes.  Called by the lanes of the halves that need it (whole halves).
__device__ int32_t half_fallback(const float *a, uint32_t M, const Stream &st)
{
    const int hl = lane_id() & 31;
    uint32_t mb = 0;
    for (uint32_t j = hl; j < M; j += 32) mb = max(mb, __float_as_uint(a[j]) & 0x7FFFFFFFu);
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) mb = max(mb, (uint32_t)__shfl_xor((int)mb, off, 32));
    const int shift = 63 - ceil_log2_u32(M) - exponent_above(__uint_as_float(mb));
    uint64_t S = 0;
    for (uint32_t j = hl; j < M; j += 32) S += fixed_weight(a[j], shift);
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) S += half_shfl_xor_u64(S, off);
    const Words w = st.block(kFallbackBlock);
    const uint64_t target = umul64hi((uint64_t)w.w0 | ((uint64_t)w.w1 << 32), S);
    uint64_t carry = 0;
    for (uint32_t base = 0; base < M; base += 32) {
        const uint32_t j = base + hl;
        const uint64_t f = j < M ? fixed_weight(a[j], shift) : 0;
        uint64_t incl = f;
#pragma unroll
        for (int d = 1; d < 32; d <<= 1) {
            const uint64_t u = half_shfl_up_u64(incl, d);
            if (hl >= d) incl += u;
        }
        incl += carry;
        const uint32_t hit = (uint32_t)(__ballot(j < M && incl > target) >> (lane_id() & 32));
        if (hit) return (int32_t)(base + __builtin_ctz(hit));
        const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)incl, 31, 32);
        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(incl >> 32), 31, 32);
        carry = (uint64_t)lo | ((uint64_t)hi << 32);
    }
    return -1;  // unreachable for S > 0
}

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_ssa_run_pair(RunArgs c)
{
    extern __shared__ int32_t lds_i[];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int h = lane >> 5, hl = lane & 31;
    const int rw = (blockIdx.x * NW + wave) * 2;
    if (rw >= c.R) return;
    const int r = rw + h;
    const bool live = r < c.R;          // the last wavefront may hold one realization
    const int N = c.net.N, M = c.net.M;
    int32_t *x = lds_i + ((size_t)wave * 2 + h) * (N + M);
    float *a = reinterpret_cast<float *>(x + N);
    int32_t *gx = c.X + (int64_t)r * N;
    if (live)
        for (int i = hl; i < N; i += 32) x[i] = gx[i];
    wave_sync_lds();
    for (int j = hl; j < M; j += 32)
        a[j] = live ? mass_action(x, c.net.r0[j], c.net.r1[j], c.net.rate[j]) : 0.0f;
    wave_sync_lds();
    const uint64_t period = max(c.period, 1u);
    const bool maintain = period > 1;
    const int L = ceil_log2_u32((uint32_t)M);
    double t = live ? c.t[r] : 0.0;
    // time steps batched as in k_ssa_run, 32 steps per half: lane hl of half
    // h holds step b0 + hl of realization r (its Philox word, and S with its
    // shift, converted at the flush); fmask bit 32 h + k marks a step that
    // fired
    uint32_t bw = 0;
    U128 bs{1, 0};
    int bsh = 0;
    uint64_t fmask = 0;
    int64_t b0 = 0;
    auto flush = [&](int64_t iend) {
        const int n = (int)(iend - b0);
        const double tau =
            ((fmask >> lane) & 1) ? neg_ln_u(bw, c.ln_tab) / wide_to_f64(bs, bsh) : 0.0;
        double tk = t;
        for (int k = 0; k < n; ++k) {
            const double t0 = readlane_f64(tau, k), t1 = readlane_f64(tau, 32 + k);
            if ((fmask >> (k + (lane & 32))) & 1) t += h ? t1 : t0;
            tk = hl == k ? t : tk;
        }
        if (c.times && live && hl < n) c.times[(b0 + hl) * c.R + r] = tk;
        fmask = 0;
        b0 = iend;
    };
    U128 S{0, 0};        // each half's alpha_0 sum (k_ssa_run)
    int Es = kNoScale;
    bool have = false;
    float B = 0.0f;
    int32_t npos = 0, nbad = 0;
    const uint32_t thresh = lemire_threshold((uint32_t)M);
    for (int64_t i = 0; i < c.steps; ++i) {
        const uint64_t s = c.step0 + (uint64_t)i;
        const bool exact = i == 0 || s % period == 0;
        if (exact) {
            uint32_t mb = 0, cnt = 0;
            for (int j = hl; j < M; j += 32) {
                const float v = a[j];
                mb = max(mb, __float_as_uint(v) & 0x7FFFFFFFu);
                cnt += (uint32_t)(v > 0.0f) + ((uint32_t)!valid_prop(v) << 16);
            }
            B = __uint_as_float(half_max_u32(mb));
            cnt = half_sum_u32(cnt);
            npos = live ? (int32_t)(cnt & 0xFFFFu) : 0;
            nbad = live ? (int32_t)(cnt >> 16) : 0;
            if (nbad == 0 && npos > 0) {
                const int e = exponent_above(B);
                if (e != Es) {
                    Es = e;
                    have = false;
                }
            } else {
                Es = kNoScale;
                have = false;
            }
        }
        // the step's selection: -2 / -1 decided, else the rounds
        int32_t j = nbad ? -2 : -1;
        bool open = live && nbad == 0 && npos > 0;
        const Stream st = make_stream(c.seed, s, (uint32_t)r, kTagSSA);
        uint32_t tau_w = 0;
        {
            const double envd = (double)B;
            uint32_t first = 0;
            bool round0 = true;
            do {
                const bool taul = round0 && hl == 31;
                const uint32_t b = taul ? kTauBlock : first + (uint32_t)hl;
                const Words w = st.block(b);
                if (round0)
                    tau_w = half_pick((uint32_t)__builtin_amdgcn_readlane((int)w.w0, 31),
                                      (uint32_t)__builtin_amdgcn_readlane((int)w.w0, 63));
                const uint64_t ta = 2 * (uint64_t)b;
                uint32_t ja = 0, jb = 0;
                const bool oka = open && !taul && lemire(w.w0, (uint32_t)M, thresh, ja) && ta < c.t_max;
                const bool okb = open && !taul && lemire(w.w2, (uint32_t)M, thresh, jb) && ta + 1 < c.t_max;
                const bool acca = oka && grid_u(w.w1) * envd < (double)a[ja];
                const bool accb = okb && grid_u(w.w3) * envd < (double)a[jb];
                const uint64_t ma = __ballot(acca), mbb = __ballot(accb);
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const uint32_t mah = (uint32_t)(ma >> (32 * hh)), mbh = (uint32_t)(mbb >> (32 * hh));
                    if (mah | mbh) {
                        const int la = mah ? __builtin_ctz(mah) : 64;
                        const int lb = mbh ? __builtin_ctz(mbh) : 64;
                        const int32_t jh = la <= lb
                            ? (int32_t)__builtin_amdgcn_readlane((int)ja, 32 * hh + la)
                            : (int32_t)__builtin_amdgcn_readlane((int)jb, 32 * hh + lb);
                        if (h == hh) {
                            j = jh;
                            open = false;
                        }
                    }
                }
                first += round0 ? 31u : 32u;
                round0 = false;
            } while (__ballot(open) && 2 * (uint64_t)first < c.t_max);
        }
        if (open) j = half_fallback(a, (uint32_t)M, st);
        if (c.fired && live && hl == 0) c.fired[i * c.R + r] = j;
        const bool fire = live && j >= 0;
        if (__ballot(fire)) {
            const int jf = fire ? j : 0;
            const int32_t nd = fire ? c.ndeps[jf] : 0;
            const int4 d0 = c.tab[(int64_t)jf * kDepMax + hl];
            const int4 d1 = c.tab[(int64_t)jf * kDepMax + 32 + hl];
            const int32_t jr0 = c.net.r0[jf], jr1 = c.net.r1[jf], jp0 = c.net.p0[jf], jp1 = c.net.p1[jf];
            if (fire && have && S.hi < (1ull << (31 - L))) {   // alpha_0 < 2^(Es-32)
                Es = kNoScale;
                have = false;
            }
            const bool need = fire && !have;
            if (__ballot(need)) {
                const bool scan = need && Es == kNoScale;
                if (__ballot(scan)) {
                    uint32_t mb = 0;
                    for (int jj = hl; jj < M; jj += 32) mb = max(mb, __float_as_uint(a[jj]) & 0x7FFFFFFFu);
                    mb = half_max_u32(mb);
                    if (scan) Es = exponent_above(__uint_as_float(mb));
                }
                const int shn = 127 - L - Es;
                U128 acc{0, 0};
                for (int jj = hl; jj < M; jj += 32)
                    acc = add128(acc, wide_weight(__float_as_uint(a[jj]), shn));
                acc = half_sum_u128(acc);
                if (need) {
                    S = acc;
                    have = true;
                }
            }
            const int sh = 127 - L - Es;
            {
                const int slot = (int)(i - b0);
                if (fire && hl == slot) {
                    bw = tau_w;
                    bs = S;
                    bsh = sh;
                }
                fmask |= __ballot(fire && hl == slot);
            }
            if (fire && hl == 0) {
                x[jr0] -= 1;
                if (jr1 >= 0) x[jr1] -= 1;
                x[jp0] += 1;
                if (jp1 >= 0) x[jp1] += 1;
            }
            wave_sync_lds();
            const bool full = fire && nd < 0;
            const uint32_t sthr = fire ? pow2_bits(Es) : 0xFFFFFFFFu;
            U128 d{0, 0};
            bool up = false;
            auto track = [&](float old, float nv) {
                d = add128(d, wide_delta(old, nv, sh));
                up |= __float_as_uint(nv) < 0x7F800000u && __float_as_uint(nv) >= sthr;
            };
            if (maintain) {
                uint32_t bm = 0;
                int32_t dpos = 0, dbad = 0;
                auto update = [&](int jj, int32_t ra, int32_t rb, float k) {
                    const float old = a[jj];
                    const float nv = mass_action(x, ra, rb, k);
                    a[jj] = nv;
                    track(old, nv);
                    if (valid_prop(nv)) bm = max(bm, __float_as_uint(nv) & 0x7FFFFFFFu);
                    dpos += (int32_t)(nv > 0.0f) - (int32_t)(old > 0.0f);
                    dbad += (int32_t)!valid_prop(nv) - (int32_t)!valid_prop(old);
                };
                if (full) {
                    for (int jj = hl; jj < M; jj += 32) update(jj, c.net.r0[jj], c.net.r1[jj], c.net.rate[jj]);
                } else if (fire) {
                    if (hl < nd) update(d0.x, d0.y, d0.z, __int_as_float(d0.w));
                    if (32 + hl < nd) update(d1.x, d1.y, d1.z, __int_as_float(d1.w));
                }
                // signed counts packed as dpos + 2^16 dbad (|sums| <= M < 2^15)
                const int32_t tot = (int32_t)half_sum_u32((uint32_t)(dpos + dbad * 65536));
                const int32_t sp = (int32_t)(int16_t)(tot & 0xFFFF);
                npos += sp;
                nbad += (tot - sp) / 65536;
                if (__ballot(bm > __float_as_uint(B))) B = fmaxf(B, __uint_as_float(half_max_u32(bm)));
            } else {
                auto update = [&](int jj, int32_t ra, int32_t rb, float k) {
                    const float old = a[jj], nv = mass_action(x, ra, rb, k);
                    a[jj] = nv;
                    track(old, nv);
                };
                if (full) {
                    for (int jj = hl; jj < M; jj += 32)
                        update(jj, c.net.r0[jj], c.net.r1[jj], c.net.rate[jj]);
                } else if (fire) {
                    if (hl < nd) update(d0.x, d0.y, d0.z, __int_as_float(d0.w));
                    if (32 + hl < nd) update(d1.x, d1.y, d1.z, __int_as_float(d1.w));
                }
            }
            // with at most 16 changes per half they sit in rows 0 and 2
            const int nmax = max(__builtin_amdgcn_readlane(nd, 0), __builtin_amdgcn_readlane(nd, 32));
            if (__ballot(full) || nmax > 16) {
                d = half_sum_u128(d);
            } else {
                d = dpp_add128<0x111>(d);
                d = dpp_add128<0x112>(d);
                d = dpp_add128<0x114>(d);
                d = dpp_add128<0x118>(d);
                const U128 s0 = readlane128(d, 15), s1 = readlane128(d, 47);
                d = (lane & 32) ? s1 : s0;
            }
            if (fire) S = add128(S, d);
            if ((uint32_t)(__ballot(up) >> (lane & 32))) {
                Es = kNoScale;
                have = false;
            }
            wave_sync_lds();
        }
        if (i + 1 - b0 == 32) flush(i + 1);
    }
    if (b0 < c.steps) flush(c.steps);
    if (live) {
        for (int i = hl; i < N; i += 32) gx[i] = x[i];
        if (hl == 0) c.t[r] = t;
    }
}

static int check_net(const arsel_network *n)
{
    if (!n || !n->r0 || !n->r1 || !n->p0 || !n->p1 || !n->rate) return ARSEL_ERR_NULL;
    if (n->N < 1 || n->M < 1) return ARSEL_ERR_SIZE;
    return ARSEL_OK;
}

static NetArgs net_args(const arsel_network *n)
{
    return NetArgs{n->r0, n->r1, n->p0, n->p1, n->rate, n->N, n->M};
}

}  // namespace arsel

using namespace arsel;

extern "C" int arsel_propensities(arsel_ctx *ctx, const arsel_network *net, const int32_t *X,
                                  int32_t R, float *alpha, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    int rc = check_net(net);
    if (rc) return rc;
    if (R < 0) return ARSEL_ERR_SIZE;
    if (R == 0) return ARSEL_OK;
    if (!X || !alpha) return ARSEL_ERR_NULL;
    if ((rc = ctx_activate(ctx))) return rc;
    const int64_t n = (int64_t)R * net->M;
    hipLaunchKernelGGL(k_propensities, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, net_args(net), X, R, alpha);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

extern "C" int arsel_ssa_chain(arsel_ctx *ctx, const arsel_network *net, int32_t *X, int32_t R,
                               uint64_t seed, uint64_t step0, int64_t steps, uint32_t t_max,
                               int64_t rec_from, int32_t *rec_X, int32_t *fired, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    int rc = check_net(net);
    if (rc) return rc;
    if (R < 0 || steps < 0 || rec_from < 0) return ARSEL_ERR_SIZE;
    if (R == 0 || steps == 0) return ARSEL_OK;
    if (!X) return ARSEL_ERR_NULL;
    if ((rc = ctx_activate(ctx))) return rc;
    const size_t per_wave = (size_t)(net->N + net->M) * 4;
    if (per_wave > ctx->lds_per_block) return ARSEL_ERR_SIZE;
    ChainArgs c{net_args(net), X, R, seed, step0, steps, t_max, rec_from, rec_X, fired};
    hipStream_t s = (hipStream_t)stream;
    if (per_wave * 4 <= ctx->tile_lds_bytes)
        hipLaunchKernelGGL(k_ssa_chain<4>, dim3((R + 3) / 4), dim3(256), per_wave * 4, s, c);
    else
        hipLaunchKernelGGL(k_ssa_chain<1>, dim3(R), dim3(64), per_wave, s, c);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

extern "C" int arsel_ssa_deps(arsel_ctx *ctx, const arsel_network *net, int32_t *deps,
                              int32_t *ndeps, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    int rc = check_net(net);
    if (rc) return rc;
    if (!deps || !ndeps) return ARSEL_ERR_NULL;
    if ((rc = ctx_activate(ctx))) return rc;
    hipLaunchKernelGGL(k_ssa_deps, dim3((net->M + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       net_args(net), deps, ndeps);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

namespace arsel {

static int ssa_run(arsel_ctx *ctx, const arsel_network *net, const int32_t *deps,
                   const int32_t *ndeps, const uint32_t *Q, int64_t ldq, uint32_t qfloor,
                   int32_t *X, int32_t R, uint64_t seed, uint64_t step0, int64_t steps,
                   uint32_t t_max, uint32_t period, double *t, double *times, int32_t *fired,
                   void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    int rc = check_net(net);
    if (rc) return rc;
    if (R < 0 || steps < 0) return ARSEL_ERR_SIZE;
    const bool prop = Q != nullptr;
    if (prop && ldq < net->M) return ARSEL_ERR_LD;
    if (R == 0 || steps == 0) return ARSEL_OK;
    if (!deps || !ndeps || !X || !t) return ARSEL_ERR_NULL;
    if ((rc = ctx_activate(ctx))) return rc;
    const size_t per_wave = (size_t)(net->N + (prop ? 2 : 1) * (size_t)net->M) * 4;
    if (per_wave > ctx->lds_per_block) return ARSEL_ERR_SIZE;
    const size_t tab_bytes = (size_t)net->M * kDepMax * sizeof(int4);
    if ((rc = ctx_grow(ctx, &ctx->ssa_tab, &ctx->ssa_tab_bytes, tab_bytes))) return rc;
    int4 *tab = (int4 *)ctx->ssa_tab;
    hipStream_t s = (hipStream_t)stream;
    const int64_t entries = (int64_t)net->M * kDepMax;
    hipLaunchKernelGGL(k_ssa_pack, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, s,
                       net_args(net), deps, ndeps, tab);
    RunArgs c{net_args(net), deps, ndeps, X, R, seed, step0, steps, t_max, t, times, fired, Q, ldq,
              qfloor, period, tab, ctx->ln_tab};
    // uniform runs with maintained envelopes: two realizations per wavefront when two
    // fit in one workgroup's LDS (and the packed counts of the exact pass fit their
    // 16-bit fields).  With period 1 the exact pass runs every step, and over 32
    // lanes it costs more than the pairing saves (measured), so one per wavefront.
    if (!prop && period > 1 && net->M < (1 << 15) && 2 * per_wave <= ctx->lds_per_block) {
        int nw = 4;
        while (nw > 1 && 2 * per_wave * nw > ctx->tile_lds_bytes) nw >>= 1;
        const int pairs = (R + 1) / 2;
        const dim3 pgrid((pairs + nw - 1) / nw), pblock(64 * nw);
        const size_t plds = 2 * per_wave * nw;
        switch (nw) {
        case 4: hipLaunchKernelGGL(k_ssa_run_pair<4>, pgrid, pblock, plds, s, c); break;
        case 2: hipLaunchKernelGGL(k_ssa_run_pair<2>, pgrid, pblock, plds, s, c); break;
        default: hipLaunchKernelGGL(k_ssa_run_pair<1>, pgrid, pblock, plds, s, c); break;
        }
        return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
    }
    // four realizations per workgroup for uniform AR; with a proposal one per
    // workgroup, whose 64-thread workgroups pack the LDS tighter (up to 15
    // against 12 realizations per CU at N = 641, M = 1029; measured 4-9%
    // faster)
    const bool four = !prop && per_wave * 4 <= ctx->tile_lds_bytes;
    const dim3 grid(four ? (R + 3) / 4 : R), block(four ? 256 : 64);
    const size_t lds = per_wave * (four ? 4 : 1);
    if (prop) {
        hipLaunchKernelGGL((k_ssa_run<1, true>), grid, block, lds, s, c);
    } else {
        if (four)
            hipLaunchKernelGGL((k_ssa_run<4, false>), grid, block, lds, s, c);
        else
            hipLaunchKernelGGL((k_ssa_run<1, false>), grid, block, lds, s, c);
    }
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

}  // namespace arsel

extern "C" int arsel_ssa_run(arsel_ctx *ctx, const arsel_network *net, const int32_t *deps,
                             const int32_t *ndeps, int32_t *X, int32_t R, uint64_t seed,
                             uint64_t step0, int64_t steps, uint32_t t_max, uint32_t period,
                             double *t, double *times, int32_t *fired, void *stream)
{
    return arsel::ssa_run(ctx, net, deps, ndeps, nullptr, 0, 0, X, R, seed, step0, steps, t_max,
                          period, t, times, fired, stream);
}

extern "C" int arsel_ssa_run_proposal(arsel_ctx *ctx, const arsel_network *net, const int32_t *deps,
                                      const int32_t *ndeps, const uint32_t *Q, int64_t ldq,
                                      uint32_t qfloor, int32_t *X, int32_t R, uint64_t seed,
                                      uint64_t step0, int64_t steps, uint32_t t_max,
                                      uint32_t period, double *t, double *times, int32_t *fired,
                                      void *stream)
{
    if (!Q) return ARSEL_ERR_NULL;
    return arsel::ssa_run(ctx, net, deps, ndeps, Q, ldq, qfloor, X, R, seed, step0, steps, t_max,
                          period, t, times, fired, stream);
}
