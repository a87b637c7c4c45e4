// Acceptance-rejection with an integer proposal Q (the learned proposal).
//
// Trial t of instance k at step s uses the tag-1 stream: its candidate word w
// gives V = hi32(w * sum Q) (rejected when lo32 < 2^32 mod sum Q, so V is
// exactly uniform on [0, sum Q)), the candidate is the least j with inclusive
// prefix P_j > V (probability Q_j / sum Q), and it is accepted when
// fl64(fl64(u c+) Q_j) < alpha_j with c+ = nextafter(max_j fl64(alpha_j / Q_j)).
// Since c+ Q_j >= alpha_j the acceptance probability is alpha_j / (c+ Q_j) up to
// the 2^-32 grid of u, so candidate-and-accept has probability proportional to
// alpha_j whatever Q is: the law stays alpha_j / alpha_0.  After t_max rejected
// trials the same fixed-point inverse transform as the uniform path runs.
#include "launch.hpp"
#include "proposal_core.hpp"

namespace arsel {

struct PropArgs {
    const float *alpha;
    const uint32_t *Q;
    int64_t lda, ldq;
    int32_t M, K;
    uint64_t seed, step;
    uint32_t t_max;
    int32_t *index;
    uint32_t *trials;
};

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_select_proposal(PropArgs a)
{
    extern __shared__ uint32_t lds_u[];
    const int wave = threadIdx.x >> 6;
    const int lane = lane_id();
    const int k = blockIdx.x * NW + wave;
    if (k >= a.K) return;
    const uint32_t M = (uint32_t)a.M;
    // per wave: alpha, then Q (replaced in place by its inclusive prefix P
    // once c is known; Q_j = P_j - P_{j-1} afterwards)
    float *sa = reinterpret_cast<float *>(lds_u) + (size_t)wave * 2 * M;
    uint32_t *sq = lds_u + (size_t)wave * 2 * M + M;
    uint32_t *sp = sq;
    const float *ga = a.alpha + (int64_t)k * a.lda;
    const uint32_t *gq = a.Q + (int64_t)k * a.ldq;

    // stage alpha and Q with vector loads (several in flight per lane); the
    // bit maximum of alpha certifies validity and is alpha_max (else an
    // exact scan decides)
    uint32_t mb = wave_max_u32(stream_bitmax<kWave>(ga, M, sa, lane));
    uint64_t sumq = 0;
    stream_each<kWave>(reinterpret_cast<const float *>(gq), M, lane, [&](uint32_t j, float x) {
        const uint32_t q = __float_as_uint(x);
        sq[j] = q;
        sumq += q;
    });
    sumq = wave_sum_u64(sumq);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float amax;
    bool bad;
    if (mb < 0x7F800000u) {
        amax = __uint_as_float(mb);
        bad = false;
    } else {
        wave_scan(ContigAcc{sa}, M, amax, bad);
    }
    bool miss = false;
    const double c = wave_proposal_c(sa, M, [&](uint32_t j) { return sq[j]; }, miss);
    Outcome o;
    o.trials = 0;
    if (bad)
        o.index = -2;
    else if (amax == 0.0f)
        o.index = -1;
    else if (miss || sumq >= (1ull << 32))
        o.index = -4;
    else {
        wave_prefix_u32([&](uint32_t j) { return sq[j]; }, sp, M);   // in place: sp aliases sq
        const double cplus = __longlong_as_double(__double_as_longlong(c) + 1);   // nextafter up
        const Stream st = make_stream(a.seed, a.step, (uint32_t)k, kTagProposal);
        o = wave_proposal_rounds(sa, sp, M, (uint32_t)sumq, cplus, amax, st, a.t_max);
    }
    if (lane == 0) {
        a.index[k] = o.index;
        if (a.trials) a.trials[k] = o.trials;
    }
}

}  // namespace arsel

using namespace arsel;

extern "C" int arsel_select_proposal(arsel_ctx *ctx, const float *alpha, const uint32_t *Q, int32_t M,
                                     int32_t K, int64_t lda, int64_t ldq, uint64_t seed, uint64_t step,
                                     uint32_t t_max, int32_t *index, uint32_t *trials, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    if (M < 1 || K < 0) return ARSEL_ERR_SIZE;
    if ((lda != 0 && lda < M) || (ldq != 0 && ldq < M)) return ARSEL_ERR_LD;
    if (K == 0) return ARSEL_OK;
    if (!alpha || !Q || !index) return ARSEL_ERR_NULL;
    int rc = ctx_activate(ctx);
    if (rc) return rc;
    if (lda == 0 && ldq == 0 && packed_lds_bytes(M, true) + 4096 <= ctx->lds_per_block)
        return launch_packed(ctx, alpha, Q, M, K, seed, step, t_max, index, nullptr, trials,
                             (hipStream_t)stream);
    const size_t per_wave = (size_t)2 * M * sizeof(uint32_t);
    int nw = 4;
    while (nw > 1 && per_wave * nw > ctx->tile_lds_bytes) nw >>= 1;
    if (per_wave * nw > ctx->lds_per_block) return ARSEL_ERR_SIZE;
    PropArgs a{alpha, Q, lda, ldq, M, K, seed, step, t_max, index, trials};
    hipStream_t s = (hipStream_t)stream;
    const int grid = (K + nw - 1) / nw;
    switch (nw) {
    case 4: hipLaunchKernelGGL(k_select_proposal<4>, dim3(grid), dim3(256), per_wave * 4, s, a); break;
    case 2: hipLaunchKernelGGL(k_select_proposal<2>, dim3(grid), dim3(128), per_wave * 2, s, a); break;
    default: hipLaunchKernelGGL(k_select_proposal<1>, dim3(grid), dim3(64), per_wave, s, a); break;
    }
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}
