// Acceptance-rejection with an integer proposal Q, one instance per
// wavefront, alpha and the inclusive prefix P of Q in LDS (shared by the
// per-instance proposal kernel and the full SSA run with a proposal).
//
// Trial t (tag-1 stream): V = Lemire draw on sum Q, j = least index with
// P_j > V (probability Q_j / sum Q), accepted when
// fl64(fl64(u c+) Q_j) < alpha_j with c+ = nextafter(max_j fl64(alpha_j / Q_j));
// since c+ Q_j >= alpha_j the selection law is alpha_j / alpha_0 for any Q
// that is positive on the support.  After t_max rejected trials the exact
// fixed-point inverse transform runs.
#pragma once

#include "select_core.hpp"
#include "wave_reduce.hpp"

namespace arsel {

// Filter estimate of alpha_j / q for q >= 1: the conversion of q, the
// hardware reciprocal (1 ulp) and the product keep its relative error below
// 2^-21 whenever the result is normal.
__device__ __forceinline__ float ratio_estimate(float x, uint32_t q)
{
    return x * __builtin_amdgcn_rcpf((float)q);
}

// c = max over the support (alpha_j > 0) of fl64(alpha_j / Q_j), Q_j = qat(j)
// > 0 there, given rmax, the wavefront maximum of the estimates over the
// support.  Rounding is monotone, so c is fl64 of the largest exact ratio;
// while rmax >= 2^-100 every index whose ratio is within 2^-20 of the largest
// has its estimate within 2^-19 of rmax, and only indices in that band get
// the binary64 division.  Tiny ratios take the exact loop over all indices.
template <class QAt>
__device__ double wave_proposal_c_band(const float *sa, uint32_t M, QAt qat, float rmax)
{
    const int lane = lane_id();
    const bool fast = rmax >= 0x1p-100f;
    const float thr = rmax - rmax * 0x1p-19f;
    double c = 0.0;
    for (uint32_t j = lane; j < M; j += kWave) {
        const float x = sa[j];
        if (x > 0.0f) {
            const uint32_t q = qat(j);
            if (q != 0 && (!fast || ratio_estimate(x, q) >= thr))
                c = fmax(c, (double)x / (double)q);
        }
    }
    return wave_max_f64_nonneg(c);
}

// The same c with its own estimate pass; miss: some alpha_j > 0 has Q_j = 0.
template <class QAt>
__device__ double wave_proposal_c(const float *sa, uint32_t M, QAt qat, bool &miss)
{
    const int lane = lane_id();
    bool ms = false;
    float rmax = 0.0f;
    for (uint32_t j = lane; j < M; j += kWave) {
        const float x = sa[j];
        if (x > 0.0f) {
            const uint32_t q = qat(j);
            if (q == 0)
                ms = true;
            else
                rmax = fmaxf(rmax, ratio_estimate(x, q));
        }
    }
    miss = __ballot(ms) != 0;
    return wave_proposal_c_band(sa, M, qat, wave_max_f32_nonneg(rmax));
}

// The rounds and the fallback for one instance: alpha in sa (valid, not all
// zero), inclusive prefix of Q in sp (S = sum Q < 2^32, every Q_j > 0 on the
// support), c+ the envelope (>= max_j alpha_j / Q_j), amax the exact maximum
// of alpha, or any value <= 0 when unknown (the fallback then scans for it).
__device__ inline Outcome wave_proposal_rounds(const float *sa, const uint32_t *sp, uint32_t M,
                                               uint32_t S, double cplus, float amax,
                                               const Stream &st, uint32_t t_max)
{
    const int lane = lane_id();
    const uint32_t thresh = lemire_threshold(S);
    const uint32_t rounds = (uint32_t)(((uint64_t)t_max + kRoundTrials - 1) / kRoundTrials);
    // least j with P_j > V for both trials of a lane: P is nondecreasing, so
    // that j is the number of P_j <= V, found by adding power-of-two steps
    // (the same number of steps in every lane; the two searches' loads are
    // independent and overlap)
    uint32_t top = 1;
    while (2 * top <= M) top *= 2;
    auto pick2 = [&](uint32_t Va, uint32_t Vb, uint32_t &ja, uint32_t &jb) {
        uint32_t pa = 0, pb = 0;
        for (uint32_t step = top; step > 0; step >>= 1) {
            const uint32_t ia = pa + step, ib = pb + step;
            const uint32_t xa = sp[min(ia, M) - 1], xb = sp[min(ib, M) - 1];
            if (ia <= M && xa <= Va) pa = ia;
            if (ib <= M && xb <= Vb) pb = ib;
        }
        ja = min(pa, M - 1);
        jb = min(pb, M - 1);
    };
    auto accept = [&](uint32_t j, uint32_t uw) {
        const double uc = grid_u(uw) * cplus;
        const uint32_t qj = sp[j] - (j ? sp[j - 1] : 0u);
        return uc * (double)qj < (double)sa[j];
    };
    Outcome o;
    o.alpha0 = 0.0f;
    uint64_t key = kNoAccept;
    for (uint32_t r = 0; r < rounds && key == kNoAccept; r = uniform_u32(r + 1)) {
        const uint64_t t0 = (uint64_t)r * kRoundTrials;
        const Words w = st.block((uint32_t)(t0 >> 1) + (uint32_t)lane);
        const uint64_t ta = t0 + 2 * (uint64_t)lane;
        uint32_t va, vb;
        const bool oka = lemire(w.w0, S, thresh, va) && ta < t_max;
        const bool okb = lemire(w.w2, S, thresh, vb) && ta + 1 < t_max;
        uint32_t ja, jb;
        pick2(va, vb, ja, jb);
        const bool acca = oka && accept(ja, w.w1);
        const bool accb = okb && accept(jb, w.w3);
        const uint64_t ma = __ballot(acca), mb = __ballot(accb);
        if (ma | mb) {
            const int la = first_lane(ma), lb = first_lane(mb);
            key = la <= lb ? ((t0 + 2 * (uint64_t)la) << 32) | readlane_u32(ja, la)
                           : ((t0 + 2 * (uint64_t)lb + 1) << 32) | readlane_u32(jb, lb);
        }
    }
    if (key != kNoAccept) {
        o.index = (int32_t)(uint32_t)key;
        o.trials = (uint32_t)(key >> 32) + 1;
    } else {
        const ContigAcc acc{sa};
        if (!(amax > 0.0f)) {
            bool bad;
            wave_scan(acc, M, amax, bad);
        }
        const int shift = 63 - ceil_log2_u32(M) - exponent_above(amax);
        const uint64_t Sf = wave_fixed_sum(acc, M, shift);
        const Words w = st.block(kFallbackBlock);
        const uint64_t V = (uint64_t)w.w0 | ((uint64_t)w.w1 << 32);
        o.index = wave_fixed_search(acc, M, shift, umul64hi(V, Sf));
        o.trials = t_max + 1;
    }
    return o;
}

// Inclusive prefix of q over [0, M) into p (may alias q; sum < 2^32): lane l
// owns the contiguous range [l per, (l + 1) per), one DPP scan of the range
// sums.  Ends with a wavefront LDS barrier.
template <class QAt>
__device__ __forceinline__ void wave_prefix_u32(QAt qat, uint32_t *p, uint32_t M)
{
    const int lane = lane_id();
    const uint32_t per = (M + kWave - 1) / kWave;
    const uint32_t lo = min((uint32_t)lane * per, M), hi = min(lo + per, M);
    uint32_t part = 0;
    for (uint32_t j = lo; j < hi; ++j) part += qat(j);
    uint32_t run = wave_incl_scan_u32(part) - part;
    for (uint32_t j = lo; j < hi; ++j) {
        run += qat(j);
        p[j] = run;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace arsel
