// The paper's own scheme (section "A GPU acceptance-rejection algorithm
// (GPU/AR) for SSA", election and selection steps), for comparison with the
// exact AR of the other kernels.
//
// Election: reaction j draws u_j = w_j 2^-32 T (binary64), T = w alpha_max,
// from word j mod 4 of Philox block j / 4 of the tag-3 stream (instance k,
// step s); it is eligible when u_j < D_j (D_j > 0) and rated R_j = u_j / D_j.
// Selection: the eligible reaction with the lowest rating (least index on
// ties); -5 when none is eligible (the paper's "M + 1").  A non-eligible
// reaction never wins (the pseudo-code's default rating 10 T could undercut
// real ratings when T < 0.1).  The paper runs one thread per reaction and a
// shared-memory tree reduction per realization; here one wavefront per
// instance evaluates four reactions per Philox block and reduces (rating,
// index) pairs with butterfly shuffles.  The law of this scheme is not
// alpha_j / alpha_0.
#include "launch.hpp"
#include "select_core.hpp"

namespace arsel {

constexpr uint32_t kTagPaper = 3;

struct PaperArgs {
    const float *alpha;
    int64_t ld;
    int32_t M, K;
    double w;
    uint64_t seed, step;
    int32_t *index;
};

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_select_paper(PaperArgs a)
{
    const int lane = lane_id();
    const int k = blockIdx.x * NW + (threadIdx.x >> 6);
    if (k >= a.K) return;
    const uint32_t M = (uint32_t)a.M;
    const float *row = a.alpha + (int64_t)k * a.ld;
    // validity and alpha_max: the bit maximum certifies a valid row
    const uint32_t mb = wave_max_u32(stream_bitmax<kWave>(row, M, nullptr, lane));
    float amax;
    bool bad;
    if (mb < 0x7F800000u) {
        amax = __uint_as_float(mb);
        bad = false;
    } else {
        wave_scan(ContigAcc{row}, M, amax, bad);
    }
    int32_t out;
    if (bad) {
        out = -2;
    } else if (amax == 0.0f) {
        out = -1;
    } else {
        const double T = a.w * (double)amax;
        const Stream st = make_stream(a.seed, a.step, (uint32_t)k, kTagPaper);
        double best_r = __builtin_inf();
        uint32_t best_j = 0xFFFFFFFFu;
        const uint32_t nb = (M + 3) >> 2;
        for (uint32_t b = lane; b < nb; b += kWave) {
            const Words wd = st.block(b);
            const uint32_t wv[4] = {wd.w0, wd.w1, wd.w2, wd.w3};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t j = 4 * b + e;
                if (j < M) {
                    const double d = (double)row[j];
                    const double u = grid_u(wv[e]) * T;
                    if (d > 0.0 && u < d) {
                        const double r = u / d;
                        if (r < best_r) {
                            best_r = r;
                            best_j = j;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double r2 = __longlong_as_double(
                (long long)shfl_xor_u64((uint64_t)__double_as_longlong(best_r), off));
            const uint32_t j2 = (uint32_t)__shfl_xor((int)best_j, off, kWave);
            if (r2 < best_r || (r2 == best_r && j2 < best_j)) {
                best_r = r2;
                best_j = j2;
            }
        }
        out = best_j == 0xFFFFFFFFu ? -5 : (int32_t)best_j;
    }
    if (lane == 0) a.index[k] = out;
}

}  // namespace arsel

using namespace arsel;

extern "C" int arsel_select_paper(arsel_ctx *ctx, const float *alpha, int32_t M, int32_t K,
                                  int64_t ld, double w, uint64_t seed, uint64_t step,
                                  int32_t *index, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    if (M < 1 || K < 0) return ARSEL_ERR_SIZE;
    if (ld != 0 && ld < M) return ARSEL_ERR_LD;
    if (!(w > 0.0) || w == __builtin_inf()) return ARSEL_ERR_ARG;
    if (K == 0) return ARSEL_OK;
    if (!alpha || !index) return ARSEL_ERR_NULL;
    int rc = ctx_activate(ctx);
    if (rc) return rc;
    PaperArgs a{alpha, ld, M, K, w, seed, step, index};
    constexpr int NW = 4;
    hipLaunchKernelGGL(k_select_paper<NW>, dim3((K + NW - 1) / NW), dim3(NW * 64), 0,
                       (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}
