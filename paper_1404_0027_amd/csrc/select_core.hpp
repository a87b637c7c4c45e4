// One instance of the acceptance-rejection selection, run by one wavefront
// or by a whole workgroup.
//
// The sequential rule (section "A GPU acceptance-rejection algorithm
// (GPU/AR) for SSA": draw j and u until u * alpha_max < alpha_j) is run W
// trials at a time: lane l of wave w handles trials t0 + 128 w + 2 l and
// t0 + 128 w + 2 l + 1, both fed by one Philox block.  Two ballots and a
// first-set-lane give the least accepted trial of the wave; with several
// waves the least over waves is taken in LDS.  The answer is therefore the
// first accepted trial of the sequential rule, whatever W is.  After t_max
// rejected trials the inverse transform of section "The Stochastic
// Simulation Algorithm" runs in exact 64-bit fixed point.
#pragma once

#include "device.hpp"

namespace arsel {

constexpr uint32_t kDebugCheckBound = 1u;

// Gather accessors: alpha_j of the current instance.
struct StridedAcc {
    const float *p;
    int64_t stride;
    __device__ __forceinline__ float operator()(uint32_t j) const { return p[(int64_t)j * stride]; }
};

struct ContigAcc {
    const float *p;
    __device__ __forceinline__ float operator()(uint32_t j) const { return p[j]; }
};

struct Outcome {
    int32_t index;
    float alpha0;
    uint32_t trials;
};

// Status after the scan; returns true when the outcome is already decided.
__device__ __forceinline__ bool decide_status(bool scanned, bool bad, float amax,
                                              const float *bound_k, uint32_t flags,
                                              float &env, Outcome &o)
{
    o.alpha0 = 0.0f;
    o.trials = 0;
    if (scanned && bad) {
        o.index = -2;
        o.alpha0 = __builtin_nanf("");
        return true;
    }
    if (bound_k) {
        env = *bound_k;
        if (!(env >= 0.0f) || env == __builtin_inff()) {
            o.index = -2;
            o.alpha0 = __builtin_nanf("");
            return true;
        }
        if (scanned && (flags & kDebugCheckBound) && amax > env) {
            o.index = -3;
            o.alpha0 = __builtin_nanf("");
            return true;
        }
        if (env == 0.0f) {
            o.index = -1;
            return true;
        }
    } else {
        env = amax;
    }
    if (scanned && amax == 0.0f) {
        o.index = -1;
        return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Wavefront version.  Every lane of the wave calls it; all return the same
// outcome.
// ---------------------------------------------------------------------------
template <class Acc>
__device__ void wave_scan(const Acc &A, uint32_t M, float &amax, bool &bad)
{
    const int lane = lane_id();
    float m = 0.0f;
    bool b = false;
    for (uint32_t j = lane; j < M; j += kWave) {
        const float x = A(j);
        b |= !(x >= 0.0f) | (x == __builtin_inff());
        m = fmaxf(m, x);
    }
    bad = __ballot(b) != 0;
    amax = wave_max(m);
}

template <class Acc>
__device__ uint64_t wave_fixed_sum(const Acc &A, uint32_t M, int shift)
{
    uint64_t s = 0;
    for (uint32_t j = lane_id(); j < M; j += kWave) s += fixed_weight(A(j), shift);
    return wave_sum_u64(s);
}

// Least j whose inclusive prefix of F exceeds target, scanning 64 at a time.
template <class Acc>
__device__ int32_t wave_fixed_search(const Acc &A, uint32_t M, int shift, uint64_t target)
{
    const int lane = lane_id();
    uint64_t carry = 0;
    for (uint32_t base = 0; base < M; base += kWave) {
        const uint32_t j = base + lane;
        const uint64_t f = j < M ? fixed_weight(A(j), shift) : 0;
        const uint64_t incl = carry + wave_incl_scan_u64(f);
        const uint64_t hit = __ballot(j < M && incl > target);
        if (hit) return (int32_t)(base + first_lane(hit));
        carry = readlane_u64(incl, kWave - 1);
    }
    return -1;  // unreachable for S > 0
}

// Result of the scan phase of one instance.
struct ScanState {
    bool decided;      // the outcome is final (-1/-2/-3)
    bool scanned;      // amax is the true maximum
    float amax;
    float env;         // envelope of the acceptance test
    Outcome o;         // final outcome when decided; alpha0 otherwise
};

template <class Acc>
__device__ ScanState wave_prepare(const Acc &A, uint32_t M, const float *bound_k, uint32_t flags,
                                  bool want_alpha0)
{
    ScanState s;
    s.scanned = (bound_k == nullptr) || (flags & kDebugCheckBound) || want_alpha0;
    s.amax = 0.0f;
    s.env = 0.0f;
    bool bad = false;
    if (s.scanned) wave_scan(A, M, s.amax, bad);
    s.decided = decide_status(s.scanned, bad, s.amax, bound_k, flags, s.env, s.o);
    if (!s.decided && s.scanned && want_alpha0) {
        const int shift = 63 - ceil_log2_u32(M) - exponent_above(s.amax);
        s.o.alpha0 = fixed_to_float(wave_fixed_sum(A, M, shift), shift);
    }
    return s;
}

constexpr uint64_t kNoAccept = ~0ull;
constexpr int kRoundTrials = 2 * kWave;   // trials per wavefront per round

// Trials [128 r, 128 r + 128) of one instance; the least accepted one packed
// as (trial << 32) | j, or kNoAccept.
template <class Acc>
__device__ __forceinline__ uint64_t wave_round(const Acc &A, uint32_t M, uint32_t thresh,
                                               double envd, const Stream &st, uint32_t r,
                                               uint32_t t_max)
{
    const int lane = lane_id();
    const uint64_t t0 = (uint64_t)r * kRoundTrials;
    const Words w = st.block((uint32_t)(t0 >> 1) + (uint32_t)lane);
    const uint64_t ta = t0 + 2 * (uint64_t)lane;
    uint32_t ja, jb;
    const bool oka = lemire(w.w0, M, thresh, ja) && ta < t_max;
    const bool okb = lemire(w.w2, M, thresh, jb) && ta + 1 < t_max;
    const bool acca = oka && grid_u(w.w1) * envd < (double)A(ja);
    const bool accb = okb && grid_u(w.w3) * envd < (double)A(jb);
    const uint64_t ma = __ballot(acca), mb = __ballot(accb);
    if ((ma | mb) == 0) return kNoAccept;
    const int la = first_lane(ma), lb = first_lane(mb);
    if (la <= lb)
        return ((t0 + 2 * (uint64_t)la) << 32) | readlane_u32(ja, la);
    return ((t0 + 2 * (uint64_t)lb + 1) << 32) | readlane_u32(jb, lb);
}

// Exact inverse-transform fallback (scans again when the scan phase was skipped).
template <class Acc>
__device__ Outcome wave_fallback(const Acc &A, uint32_t M, bool scanned, float amax,
                                 const Stream &st, uint32_t t_max, float alpha0)
{
    Outcome o;
    o.alpha0 = alpha0;
    o.trials = 0;
    if (!scanned) {
        bool bad = false;
        wave_scan(A, M, amax, bad);
        if (bad) {
            o.index = -2;
            return o;
        }
        if (amax == 0.0f) {
            o.index = -1;
            return o;
        }
    }
    const int shift = 63 - ceil_log2_u32(M) - exponent_above(amax);
    const uint64_t S = wave_fixed_sum(A, M, shift);
    const Words w = st.block(kFallbackBlock);
    const uint64_t V = (uint64_t)w.w0 | ((uint64_t)w.w1 << 32);
    o.index = wave_fixed_search(A, M, shift, umul64hi(V, S));
    o.trials = t_max + 1;
    return o;
}

// Rounds and fallback of one instance whose scan phase is done.
template <class Acc>
__device__ Outcome wave_run(const Acc &A, uint32_t M, const ScanState &s, const Stream &st,
                            uint32_t t_max)
{
    if (s.decided) return s.o;
    const uint32_t thresh = lemire_threshold(M);
    const double envd = (double)s.env;
    const uint32_t rounds = (uint32_t)(((uint64_t)t_max + kRoundTrials - 1) / kRoundTrials);
    for (uint32_t r = 0; r < rounds; ++r) {
        const uint64_t key = wave_round(A, M, thresh, envd, st, r, t_max);
        if (key != kNoAccept) {
            Outcome o = s.o;
            o.index = (int32_t)(uint32_t)key;
            o.trials = (uint32_t)(key >> 32) + 1;
            return o;
        }
    }
    return wave_fallback(A, M, s.scanned, s.amax, st, t_max, s.o.alpha0);
}

template <class Acc>
__device__ Outcome wave_select(const Acc &A, uint32_t M, const float *bound_k, uint32_t flags,
                               const Stream &st, uint32_t t_max, bool want_alpha0)
{
    return wave_run(A, M, wave_prepare(A, M, bound_k, flags, want_alpha0), st, t_max);
}

// As wave_select without a bound, given the bit-maximum of the instance taken
// while it was loaded: below 0x7F800000 it certifies a valid vector and is
// alpha_max itself, so the scan is skipped; otherwise the exact scan runs.
template <class Acc>
__device__ Outcome wave_select_hint(const Acc &A, uint32_t M, uint32_t maxbits, const Stream &st,
                                    uint32_t t_max, bool want_alpha0)
{
    if (maxbits >= 0x7F800000u) return wave_select(A, M, nullptr, 0u, st, t_max, want_alpha0);
    ScanState s;
    s.scanned = true;
    s.amax = __uint_as_float(maxbits);
    s.decided = decide_status(true, false, s.amax, nullptr, 0u, s.env, s.o);
    if (!s.decided && want_alpha0) {
        const int shift = 63 - ceil_log2_u32(M) - exponent_above(s.amax);
        s.o.alpha0 = fixed_to_float(wave_fixed_sum(A, M, shift), shift);
    }
    return wave_run(A, M, s, st, t_max);
}

// Stream n floats from src (4-byte aligned) with 16-byte loads, kStreamBatch
// per thread in flight; thread tid of NT takes every NT-th slot and calls
// f(j, alpha_j) for each element it loads (any order).
constexpr int kStreamBatch = 8;

template <int NT, class F>
__device__ __forceinline__ void stream_each(const float *src, uint32_t n, int tid, F &&f)
{
    const uint32_t align = (uint32_t)(((16 - ((uintptr_t)src & 15)) & 15) >> 2);
    const uint32_t head = align < n ? align : n;
    if ((uint32_t)tid < head) f((uint32_t)tid, src[tid]);
    const uint32_t nq = (n - head) >> 2;
    const float *s4 = src + head;
    for (uint32_t base = 0; base < nq; base += kStreamBatch * NT) {
        f32x4 v[kStreamBatch];
#pragma unroll
        for (int u = 0; u < kStreamBatch; ++u) {
            const uint32_t i = base + u * NT + tid;
            if (i < nq) v[u] = load_stream4(s4 + 4 * i);
        }
#pragma unroll
        for (int u = 0; u < kStreamBatch; ++u) {
            const uint32_t i = base + u * NT + tid;
            if (i < nq) {
                const uint32_t j = head + 4 * i;
                f(j, v[u].x);
                f(j + 1, v[u].y);
                f(j + 2, v[u].z);
                f(j + 3, v[u].w);
            }
        }
    }
    for (uint32_t j = head + 4 * nq + tid; j < n; j += NT) f(j, src[j]);
}

// Streaming pass that copies the elements to dst (LDS) when dst is not null
// and returns the thread's running maximum of the raw bits (the certificate
// used by wave_select_hint).
template <int NT>
__device__ __forceinline__ uint32_t stream_bitmax(const float *src, uint32_t n, float *dst, int tid)
{
    uint32_t mb = 0;
    if (dst)
        stream_each<NT>(src, n, tid, [&](uint32_t j, float x) {
            mb = max(mb, __float_as_uint(x));
            dst[j] = x;
        });
    else
        stream_each<NT>(src, n, tid, [&](uint32_t, float x) { mb = max(mb, __float_as_uint(x)); });
    return mb;
}

// The thread's part of sum_j floor(alpha_j 2^shift) over a global row.
template <int NT>
__device__ __forceinline__ uint64_t stream_fixed_sum(const float *src, uint32_t n, int shift, int tid)
{
    uint64_t s = 0;
    stream_each<NT>(src, n, tid, [&](uint32_t, float x) { s += fixed_weight(x, shift); });
    return s;
}

}  // namespace arsel
