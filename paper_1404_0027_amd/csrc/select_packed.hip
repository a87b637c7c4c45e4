// Broadcast selection with packed rounds: K selections from ONE propensity
// vector (uniform proposal) or one (alpha, Q) pair (integer proposal).
//
// The vector is staged in LDS once per workgroup.  A wavefront then serves
// 64 / L instances at a time, L lanes per instance: in round r, lane l of an
// instance's group evaluates Philox block r L + l of that instance's stream,
// i.e. trials 2(r L + l) and 2(r L + l) + 1 -- exactly the trials the
// one-wavefront kernels evaluate -- and the least accepted trial of the
// group's round wins (ballot, then first set lane of the group).  Rounds of
// an instance run in increasing order, so the answer is the sequential rule's
// (section "A GPU acceptance-rejection algorithm (GPU/AR) for SSA": the first
// accepted draw) for every L: the trial width is a schedule parameter.
//
// Each trial costs one half Philox block whatever L is; a wide group wastes
// the trials after the first accepted one in its round, a narrow one spends
// more rounds, hands out instances more often and waits longer for the last
// one of a workgroup.  With one lane per instance (L = 1) no trial is wasted
// beyond the accepted one and its twin, so the Philox work per selection is
// about 1 / (2 p) blocks for per-trial acceptance p -- the width a proposal
// close to alpha / alpha_0 (p near 1) runs at.  For small p the automatic
// width grows to about 1 / (2 p) lanes (the expected trials of a selection
// in one round); for small K it grows until every lane has an instance.
#include "launch.hpp"
#include "select_block.hpp"
#include "wave_reduce.hpp"

namespace arsel {

struct PackedArgs {
    const float *alpha;      // [M]
    const uint32_t *Q;       // [M] (proposal mode) or null (uniform mode)
    int32_t M, K;
    uint64_t seed, step;
    uint32_t t_max;
    int32_t *index;
    float *alpha0;           // uniform mode only (nullable)
    uint32_t *trials;        // nullable
    int32_t lanes;           // L (power of two, 1..64), 0: chosen in the kernel
    int32_t per_block;       // instances per workgroup
    int32_t fill_lanes;      // L that would give every lane of the launch an instance
};

template <int NW>
__device__ __forceinline__ uint64_t block_max_u64(uint64_t x, BlockScratch<NW> &bs)
{
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t o = shfl_xor_u64(x, off);
        x = o > x ? o : x;
    }
    if (lane_id() == 0) bs.red64[wave] = x;
    __syncthreads();
    uint64_t m = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) m = bs.red64[w] > m ? bs.red64[w] : m;
    __syncthreads();
    return m;
}

// Least j with P_j > V over the inclusive prefix P (LDS), P_{M-1} > V, by a
// guide table (the cutpoint method of Chen and Asau): G[b] is the least j with
// P_j > b 2^gs, a lower bound of the answer for every V in [b 2^gs,
// (b + 1) 2^gs), from which a forward scan reaches the answer exactly.  With
// about one reaction per bucket the scan takes one or two steps.
__device__ __forceinline__ uint32_t guide_pick(const uint32_t *P, const uint32_t *G, uint32_t gs,
                                               uint32_t V)
{
    uint32_t j = G[(uint32_t)((uint64_t)V >> gs)];   // gs may be 32 (M = 1)
    while (P[j] <= V) ++j;
    return j;
}

struct PackedShared {
    uint32_t cursor;
    int32_t status;          // 0: run trials; < 0: the outcome of every instance
    uint32_t lanes_log2;
    uint32_t sumq;
    uint32_t gs;             // guide-table bucket width log2
    float amax;
    float alpha0;
    double env;              // alpha_max (uniform) or c+ (proposal)
};

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_select_packed(PackedArgs a)
{
    extern __shared__ uint32_t lds_u[];
    __shared__ BlockScratch<NW> bs;
    __shared__ PackedShared sh;
    constexpr int NT = NW * kWave;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const uint32_t M = (uint32_t)a.M;
    const bool prop = a.Q != nullptr;
    float *sa = reinterpret_cast<float *>(lds_u);
    uint32_t *sq = lds_u + M;        // proposal: Q
    uint32_t *sp = lds_u + 2 * M;    // proposal: inclusive prefix of Q
    uint32_t *sg = lds_u + 3 * M;    // proposal: guide table (2^ceil(log2 M) entries)
    const int k_lo = blockIdx.x * a.per_block;
    const int k_hi = min(a.K, k_lo + a.per_block);

    // ---- stage and classify (once per workgroup) ----
    uint32_t mb = stream_bitmax<NT>(a.alpha, M, sa, tid);
    uint64_t sumq = 0;
    if (prop)
        for (uint32_t j = tid; j < M; j += NT) {
            const uint32_t q = a.Q[j];
            sq[j] = q;
            sumq += q;
        }
    mb = block_max_u32<NW>(mb, bs);   // its barriers also publish the staged arrays
    float amax;
    bool bad;
    if (mb < 0x7F800000u) {
        amax = __uint_as_float(mb);
        bad = false;
    } else {
        block_scan<NW>(ContigAcc{sa}, M, amax, bad, bs);
    }
    int32_t status = bad ? -2 : (amax == 0.0f ? -1 : 0);
    const int L2 = ceil_log2_u32(M);
    const int shift = status == 0 ? 63 - L2 - exponent_above(amax) : 0;
    double env = (double)amax;
    double phat = 0.0;
    float alpha0 = status == -2 ? __builtin_nanf("") : 0.0f;
    if (status == 0) {
        uint64_t s = 0;
        for (uint32_t j = tid; j < M; j += NT) s += fixed_weight(sa[j], shift);
        const uint64_t S = block_sum_u64<NW>(s, bs);
        alpha0 = fixed_to_float(S, shift);
        const double a0 = ldexp((double)S, -shift);
        if (prop) {
            // support covered, sum Q < 2^32, c = max fl64(alpha_j / Q_j), prefix
            uint64_t cbits = 0;
            uint32_t miss = 0;
            for (uint32_t j = tid; j < M; j += NT) {
                const float x = sa[j];
                if (x > 0.0f) {
                    const uint32_t q = sq[j];
                    if (q == 0) {
                        miss = 1;
                    } else {
                        const uint64_t b = (uint64_t)__double_as_longlong((double)x / (double)q);
                        cbits = b > cbits ? b : cbits;
                    }
                }
            }
            miss = block_max_u32<NW>(miss, bs);
            const uint64_t SQ = block_sum_u64<NW>(sumq, bs);
            cbits = block_max_u64<NW>(cbits, bs);
            if (miss || SQ >= (1ull << 32)) {
                status = -4;
            } else {
                // inclusive prefix: thread i owns a contiguous range
                const uint32_t per = (M + NT - 1) / NT;
                const uint32_t lo = min((uint32_t)tid * per, M), hi = min(lo + per, M);
                uint64_t part = 0;
                for (uint32_t j = lo; j < hi; ++j) part += sq[j];
                uint64_t tot;
                uint64_t run = block_excl_scan_u64<NW>(part, tot, bs);
                for (uint32_t j = lo; j < hi; ++j) {
                    run += sq[j];
                    sp[j] = (uint32_t)run;
                }
                // guide table: buckets of width 2^gs, at most 2^ceil(log2 M) of them
                const int bits = 64 - __clzll((long long)SQ);
                const uint32_t gs = (uint32_t)max(0, bits - L2);
                __syncthreads();
                for (uint32_t j = lo; j < hi; ++j) {
                    const uint64_t prev = j == 0 ? 0ull : (uint64_t)sp[j - 1];
                    const uint64_t cur = (uint64_t)sp[j];
                    const uint64_t b0 = (prev + (1ull << gs) - 1) >> gs;
                    const uint64_t b1 = (cur + (1ull << gs) - 1) >> gs;
                    for (uint64_t b = b0; b < b1; ++b) sg[b] = j;
                }
                env = __longlong_as_double((long long)(cbits + 1));   // c+ = nextafter(c, +inf)
                phat = a0 / (env * (double)SQ);
                if (tid == 0) {
                    sh.sumq = (uint32_t)SQ;
                    sh.gs = gs;
                }
            }
        } else {
            phat = a0 / ((double)M * (double)amax);
        }
    }
    if (tid == 0) {
        sh.status = status;
        sh.amax = amax;
        sh.alpha0 = alpha0;
        sh.env = env;
        sh.cursor = (uint32_t)k_lo;
        // trial width: as given, else as wide as the expected trials per
        // selection (1 / p) use, and at least as wide as gives every lane of
        // the launch an instance (measured: with 2^20 uniform-AR instances,
        // p ~ 0.05, 8 lanes per instance run 2x faster than 1 -- fewer
        // instance hand-offs and a shorter tail per round of trials)
        int l2 = 0;
        if (a.lanes > 0) {
            l2 = 31 - __clz(a.lanes);
        } else if (status == 0) {
            const double want = phat > 0.0 ? 0.5 / phat : 64.0;
            while (l2 < 6 && ((double)(2 << l2) <= want || (1 << (l2 + 1)) <= a.fill_lanes)) ++l2;
        }
        sh.lanes_log2 = (uint32_t)l2;
    }
    __syncthreads();
    status = sh.status;

    if (status != 0) {
        for (int k = k_lo + tid; k < k_hi; k += NT) {
            a.index[k] = status;
            if (a.alpha0) a.alpha0[k] = status == -1 ? 0.0f : __builtin_nanf("");
            if (a.trials) a.trials[k] = 0;
        }
        return;
    }

    // ---- packed rounds ----
    const uint32_t l2 = uniform_u32(sh.lanes_log2);
    const uint32_t Lw = 1u << l2;                           // lanes per instance
    const uint32_t g = (uint32_t)lane >> l2;                 // my group
    const uint32_t gl = (uint32_t)lane & (Lw - 1);           // my lane in the group
    const uint32_t gbase = g << l2;
    const uint64_t gmask = Lw == 64 ? ~0ull : ((1ull << Lw) - 1);
    const double envd = sh.env;
    const uint32_t SQ = prop ? sh.sumq : 0u;
    const uint32_t gs = prop ? sh.gs : 0u;
    const uint32_t nq = prop ? SQ : M;
    const uint32_t thresh = lemire_threshold(nq);
    const uint64_t tmax = a.t_max;
    const uint32_t tag = prop ? kTagProposal : kTagUniform;
    const float a0_out = sh.alpha0;
    const float amax_u = sh.amax;

    int32_t inst = -1;          // this group's instance (-1: none)
    uint32_t r = 0;             // its next round
    bool exhausted = false;     // the workgroup's range is used up (wave-uniform)
    for (;;) {
        // hand new instances to idle groups, in group order
        const uint64_t lead = __ballot(gl == 0 && inst < 0);
        if (!exhausted && lead != 0) {
            const uint32_t want = (uint32_t)__popcll(lead);
            const uint32_t base = wave_claim_add(&sh.cursor, want);
            if (base + want >= (uint32_t)k_hi) exhausted = true;
            if (inst < 0) {
                const uint32_t rank = (uint32_t)__popcll(lead & ((1ull << gbase) - 1));
                const uint32_t k = base + rank;
                if (k < (uint32_t)k_hi) {
                    inst = (int32_t)k;
                    r = 0;
                }
            }
        }
        if (__ballot(inst >= 0) == 0) break;

        // one round of every busy group
        const bool busy = inst >= 0 && (uint64_t)r * 2 * Lw < tmax;
        const Stream st = make_stream(a.seed, a.step, (uint32_t)(inst < 0 ? 0 : inst), tag);
        const uint32_t b = r * Lw + gl;
        const uint64_t ta = 2 * (uint64_t)b;
        uint32_t ja = 0, jb = 0;
        bool acca = false, accb = false;
        if (busy) {
            const Words w = st.block(b);
            uint32_t va, vb;
            const bool oka = lemire(w.w0, nq, thresh, va) && ta < tmax;
            const bool okb = lemire(w.w2, nq, thresh, vb) && ta + 1 < tmax;
            if (prop) {
                ja = guide_pick(sp, sg, gs, va);
                jb = guide_pick(sp, sg, gs, vb);
                acca = oka && (grid_u(w.w1) * envd) * (double)sq[ja] < (double)sa[ja];
                accb = okb && (grid_u(w.w3) * envd) * (double)sq[jb] < (double)sa[jb];
            } else {
                ja = va;
                jb = vb;
                acca = oka && grid_u(w.w1) * envd < (double)sa[ja];
                accb = okb && grid_u(w.w3) * envd < (double)sa[jb];
            }
        }
        const uint64_t ma = __ballot(acca), mbb = __ballot(accb);
        const uint64_t gma = (ma >> gbase) & gmask, gmb = (mbb >> gbase) & gmask;
        const uint32_t la = gma ? (uint32_t)__builtin_ctzll(gma) : 64u;
        const uint32_t lb = gmb ? (uint32_t)__builtin_ctzll(gmb) : 64u;
        const bool use_a = la <= lb;
        const int src = (int)(gbase + (use_a ? (la & 63u) : (lb & 63u)));
        const uint32_t ja_s = (uint32_t)__shfl((int)ja, src, kWave);
        const uint32_t jb_s = (uint32_t)__shfl((int)jb, src, kWave);
        if (busy && (gma | gmb) != 0) {
            if (gl == 0) {
                const uint64_t t = use_a ? 2 * ((uint64_t)r * Lw + la) : 2 * ((uint64_t)r * Lw + lb) + 1;
                a.index[inst] = (int32_t)(use_a ? ja_s : jb_s);
                if (a.alpha0) a.alpha0[inst] = a0_out;
                if (a.trials) a.trials[inst] = (uint32_t)(t + 1);
            }
            inst = -1;
        } else if (inst >= 0) {
            ++r;
        }

        // groups whose trial budget is spent: exact fixed-point inverse
        // transform, one instance at a time with the whole wavefront
        const bool spent = inst >= 0 && (uint64_t)r * 2 * Lw >= tmax;
        uint64_t fb = __ballot(gl == 0 && spent);
        while (fb) {
            const int ld = (int)__builtin_ctzll(fb);
            fb &= fb - 1;
            const int32_t k = (int32_t)readlane_u32((uint32_t)inst, ld);
            const Stream sk = make_stream(a.seed, a.step, (uint32_t)k, tag);
            const Outcome o = wave_fallback(ContigAcc{sa}, M, true, amax_u, sk, a.t_max, a0_out);
            if (lane == 0) {
                a.index[k] = o.index;
                if (a.alpha0) a.alpha0[k] = a0_out;
                if (a.trials) a.trials[k] = o.trials;
            }
        }
        if (spent) inst = -1;
    }
}

}  // namespace arsel

using namespace arsel;

namespace arsel {

// Launch for K instances from one vector (Q null: uniform mode).
int launch_packed(arsel_ctx *ctx, const float *alpha, const uint32_t *Q, int32_t M, int32_t K,
                  uint64_t seed, uint64_t step, uint32_t t_max, int32_t *index, float *alpha0,
                  uint32_t *trials, hipStream_t s)
{
    constexpr int NW = 4;
    const size_t lds = packed_lds_bytes(M, Q != nullptr);
    if (lds > ctx->lds_per_block - 4096) return ARSEL_ERR_SIZE;
    PackedArgs a;
    a.alpha = alpha;
    a.Q = Q;
    a.M = M;
    a.K = K;
    a.seed = seed;
    a.step = step;
    a.t_max = t_max;
    a.index = index;
    a.alpha0 = Q ? nullptr : alpha0;
    a.trials = trials;
    a.lanes = ctx->trial_lanes;
    // workgroups: each stages the vector once; the proposal's longer set-up
    // (prefix, guide table, c) is amortised over more instances (about 4
    // workgroups per CU), the uniform mode gains from more resident waves (8)
    const int64_t slots = (int64_t)ctx->num_cu * (Q ? 4 : 8);
    int64_t per = ((int64_t)K + slots - 1) / slots;
    per = std::max<int64_t>(per, 64);
    a.per_block = (int32_t)per;
    const int grid = (int)(((int64_t)K + per - 1) / per);
    // lanes per instance that would still give every lane of the launch an instance
    const int64_t lanes_total = (int64_t)grid * NW * kWave;
    int fill = 1;
    while (fill < 64 && (int64_t)K * fill * 2 <= lanes_total) fill *= 2;
    a.fill_lanes = fill;
    hipLaunchKernelGGL(k_select_packed<NW>, dim3(grid), dim3(NW * kWave), lds, s, a);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

}  // namespace arsel

extern "C" int arsel_set_trial_lanes(arsel_ctx *ctx, int32_t lanes)
{
    if (!ctx) return ARSEL_ERR_NULL;
    if (lanes < 0 || lanes > 64 || (lanes & (lanes - 1)) != 0) return ARSEL_ERR_ARG;
    ctx->trial_lanes = lanes;
    return ARSEL_OK;
}
