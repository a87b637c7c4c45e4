// One instance of the acceptance-rejection selection run by a whole
// workgroup of NW wavefronts (large M).  Same rule and same random stream as
// the wavefront version: round r of the workgroup covers trials
// [128 NW r, 128 NW (r + 1)); wave w takes the 128-trial slice r NW + w and the
// least accepted trial over the waves wins, so the answer is the sequential
// rule's for any NW.
#pragma once

#include "select_core.hpp"

namespace arsel {

template <int NW>
struct BlockScratch {
    uint32_t red32[NW];
    uint64_t red64[NW];
    uint64_t key;
    int32_t found;
};

template <int NW>
__device__ __forceinline__ uint32_t block_max_u32(uint32_t x, BlockScratch<NW> &bs)
{
    const int wave = threadIdx.x >> 6;
    x = wave_max_u32(x);
    if (lane_id() == 0) bs.red32[wave] = x;
    __syncthreads();
    x = wave_max_u32(lane_id() < NW ? bs.red32[lane_id()] : 0u);
    __syncthreads();
    return x;
}

template <int NW>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t x, BlockScratch<NW> &bs)
{
    const int wave = threadIdx.x >> 6;
    x = wave_sum_u64(x);
    if (lane_id() == 0) bs.red64[wave] = x;
    __syncthreads();
    x = wave_sum_u64(lane_id() < NW ? bs.red64[lane_id()] : 0ull);
    __syncthreads();
    return x;
}

// Exclusive prefix over the threads of the block (thread order), and the total.
template <int NW>
__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t x, uint64_t &total,
                                                        BlockScratch<NW> &bs)
{
    const int wave = threadIdx.x >> 6;
    const uint64_t incl = wave_incl_scan_u64(x);
    if (lane_id() == kWave - 1) bs.red64[wave] = incl;
    __syncthreads();
    uint64_t before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint64_t v = bs.red64[w];
        if (w < wave) before += v;
        total += v;
    }
    __syncthreads();
    return before + incl - x;
}

// Scan with validation and exact maximum over the block.
template <int NW, class Acc>
__device__ void block_scan(const Acc &A, uint32_t M, float &amax, bool &bad, BlockScratch<NW> &bs)
{
    float m = 0.0f;
    uint32_t b = 0;
    for (uint32_t j = threadIdx.x; j < M; j += NW * kWave) {
        const float x = A(j);
        b |= (!(x >= 0.0f) | (x == __builtin_inff())) ? 1u : 0u;
        m = fmaxf(m, x);
    }
    // fmaxf-maximum of non-negative values: compare as bits
    const uint32_t mb = block_max_u32<NW>(__float_as_uint(m) & 0x7FFFFFFFu, bs);
    bad = block_max_u32<NW>(b, bs) != 0;
    amax = __uint_as_float(mb);
}

// Least j in [0, n) whose inclusive prefix of F_j = floor(alpha_j 2^shift)
// exceeds target, or -1 when the n elements sum to at most target.  Thread i
// owns the contiguous range [i L, (i + 1) L); range sums are read in a skewed
// order (the sum does not depend on it) so that LDS lanes do not share a bank.
// `total` returns the sum of the n weights.
template <int NW, class Acc>
__device__ int32_t block_prefix_search(const Acc &A, uint32_t n_all, int shift, uint64_t target,
                                       uint64_t &total, BlockScratch<NW> &bs)
{
    constexpr int NT = NW * kWave;
    const uint32_t tid = threadIdx.x;
    const uint32_t L = (n_all + NT - 1) / NT;
    const uint32_t lo = min(tid * L, n_all), hi = min(lo + L, n_all);
    const uint32_t n = hi - lo;
    uint64_t part = 0;
    uint32_t idx = n ? tid % n : 0;
    for (uint32_t i = 0; i < n; ++i) {
        part += fixed_weight(A(lo + idx), shift);
        idx = idx + 1 == n ? 0 : idx + 1;
    }
    uint64_t S = 0;
    const uint64_t before = block_excl_scan_u64<NW>(part, S, bs);
    total = S;
    if (tid == 0) bs.found = -1;
    __syncthreads();
    if (n > 0 && before <= target && target < before + part) {
        uint64_t P = before;
        for (uint32_t j = lo; j < hi; ++j) {
            P += fixed_weight(A(j), shift);
            if (P > target) {
                bs.found = (int32_t)j;
                break;
            }
        }
    }
    __syncthreads();
    const int32_t j = bs.found;
    __syncthreads();
    return j;
}

// Exact fixed-point inverse transform over the block (instance resident in
// LDS, or any accessor for moderate M).
template <int NW, class Acc>
__device__ int32_t block_fallback_pick(const Acc &A, uint32_t M, int shift, const Stream &st,
                                       BlockScratch<NW> &bs)
{
    // S first (the target depends on it), then the search.
    uint64_t S = 0;
    for (uint32_t j = threadIdx.x; j < M; j += NW * kWave) S += fixed_weight(A(j), shift);
    S = block_sum_u64<NW>(S, bs);
    const Words w = st.block(kFallbackBlock);
    const uint64_t V = (uint64_t)w.w0 | ((uint64_t)w.w1 << 32);
    uint64_t tot;
    return block_prefix_search<NW>(A, M, shift, umul64hi(V, S), tot, bs);
}

// The same for an instance left in global memory: one streaming pass for S,
// then the row is copied into LDS piece by piece (coalesced, several loads in
// flight) until the piece holding the target is found and searched there.
template <int NW>
__device__ int32_t block_fallback_global(const float *row, uint32_t M, int shift, const Stream &st,
                                         float *piece_buf, uint32_t piece, BlockScratch<NW> &bs)
{
    constexpr int NT = NW * kWave;
    const uint64_t S = block_sum_u64<NW>(stream_fixed_sum<NT>(row, M, shift, threadIdx.x), bs);
    const Words w = st.block(kFallbackBlock);
    const uint64_t V = (uint64_t)w.w0 | ((uint64_t)w.w1 << 32);
    const uint64_t target = umul64hi(V, S);
    uint64_t before = 0;
    for (uint32_t p0 = 0; p0 < M; p0 += piece) {
        const uint32_t n = min(piece, M - p0);
        stream_each<NT>(row + p0, n, threadIdx.x, [&](uint32_t j, float x) { piece_buf[j] = x; });
        __syncthreads();
        uint64_t part;
        const int32_t j = block_prefix_search<NW>(ContigAcc{piece_buf}, n, shift, target - before, part, bs);
        if (j >= 0) return (int32_t)p0 + j;
        before += part;
    }
    return -1;   // unreachable for S > 0
}

// The whole selection for one instance.  maxbits_hint: the block-wide bit
// maximum from a fused load pass (certifies validity when < 0x7F800000), or
// 0xFFFFFFFF when no such pass ran.
//
// global_row: the instance's row in global memory when A reads it there (no
// LDS copy); its fallback and alpha0 passes then stream the row and stage it
// piece by piece in piece_buf (piece floats).  Null when A reads LDS.
template <int NW, class Acc>
__device__ Outcome block_select(const Acc &A, uint32_t M, uint32_t maxbits_hint, const Stream &st,
                                uint32_t t_max, bool want_alpha0, BlockScratch<NW> &bs,
                                const float *global_row = nullptr, float *piece_buf = nullptr,
                                uint32_t piece = 0)
{
    const int wave = threadIdx.x >> 6;
    float amax;
    bool bad;
    if (maxbits_hint < 0x7F800000u) {
        amax = __uint_as_float(maxbits_hint);
        bad = false;
    } else {
        block_scan<NW>(A, M, amax, bad, bs);
    }
    Outcome o;
    float env = 0.0f;
    if (decide_status(true, bad, amax, nullptr, 0u, env, o)) return o;
    const int L = ceil_log2_u32(M);
    const int shift = 63 - L - exponent_above(amax);
    if (want_alpha0) {
        uint64_t s = 0;
        if (global_row)
            s = stream_fixed_sum<NW * kWave>(global_row, M, shift, threadIdx.x);
        else
            for (uint32_t j = threadIdx.x; j < M; j += NW * kWave) s += fixed_weight(A(j), shift);
        o.alpha0 = fixed_to_float(block_sum_u64<NW>(s, bs), shift);
    }
    const uint32_t thresh = lemire_threshold(M);
    const double envd = (double)env;
    const uint32_t wrounds = (uint32_t)(((uint64_t)t_max + kRoundTrials - 1) / kRoundTrials);
    for (uint32_t r0 = 0; r0 < wrounds; r0 += NW) {
        if (threadIdx.x == 0) bs.key = kNoAccept;
        __syncthreads();
        const uint32_t r = r0 + (uint32_t)wave;
        if (r < wrounds) {
            const uint64_t key = wave_round(A, M, thresh, envd, st, r, t_max);
            if (key != kNoAccept && lane_id() == 0)
                atomicMin((unsigned long long *)&bs.key, (unsigned long long)key);
        }
        __syncthreads();
        const uint64_t key = bs.key;
        __syncthreads();
        if (key != kNoAccept) {
            o.index = (int32_t)(uint32_t)key;
            o.trials = (uint32_t)(key >> 32) + 1;
            return o;
        }
    }
    if (global_row && piece_buf && piece > 0)
        o.index = block_fallback_global<NW>(global_row, M, shift, st, piece_buf, piece, bs);
    else
        o.index = block_fallback_pick<NW>(A, M, shift, st, bs);
    o.trials = t_max + 1;
    return o;
}

}  // namespace arsel
