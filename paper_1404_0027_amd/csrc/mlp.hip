// Learned proposal: a small BF16 MLP on MFMA (FP32 accumulation) that maps
// species counts to a proposal q over reactions, its integer quantisation Q,
// and its training (forward, cross-entropy gradient, backward GEMMs, Adam).
//
// Acceptance-rejection stays exact with ANY proposal that covers the support:
// a candidate j drawn with probability Q_j / sum Q is accepted with
// probability alpha_j / (c+ Q_j), c+ >= max alpha_j / Q_j, so the network only
// changes the acceptance rate, never the selection law.
//
// Network: f = bf16(log1p(X)) (N inputs, zero-padded to Kp), h1 = relu(W1 f + b1),
// h2 = relu(W2 h1 + b2), z = W3 h2 + b3 (M outputs, padded to Mp); q = softmax(z)
// over the reactions with alpha_j > 0; Q_j = max(1, floor(q_j 2^(31-L))) on
// that support (L = ceil(log2 M)), 0 elsewhere, so sum Q < 2^32.
#include <math.h>

#include "launch.hpp"
#include "device.hpp"

namespace arsel {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4m __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM: C[m][n] = sum_k A(m, k) B(n, k), BF16 inputs, FP32 accumulation on
// v_mfma_f32_16x16x32_bf16.  A(m,k) = A[m*lda + k] when A_KC (k contiguous)
// else A[k*lda + m]; B(n,k) = B[n*ldb + k] when B_KC else B[k*ldb + n].
// Workgroup tile 64 x 64, 4 wavefronts of 32 x 32 (2 x 2 MFMA blocks), K step
// 32.  Each thread moves one 16-byte chunk (8 BF16) of each operand tile per
// step; the next step's chunks are loaded into registers while the MFMAs of
// the current step run.  With grid.z > 1 the K range is split into grid.z
// slices of kslice (a multiple of the k step) and slice z writes its partial product
// to C + z * M * ldc (summed afterwards in slice order); the epilogue then
// runs in the reduction.  Epilogue: + bias[n], ReLU, zero where
// mask(m, n) <= 0, FP32 and/or BF16 out.
// ---------------------------------------------------------------------------
struct GemmArgs {
    const __bf16 *A;
    const __bf16 *B;
    int64_t lda, ldb;
    int32_t M, N, K;
    int32_t kslice;           // K range per grid.z slice (multiple of the k step)
    int32_t vec_a, vec_b;     // 16-byte chunks allowed (aligned base, ld % 8 == 0)
    const float *bias;        // [N] or null
    const __bf16 *mask;       // [M][ldm] or null
    int64_t ldm;
    float *C;                 // [M][ldc] or null
    int64_t ldc;
    __bf16 *Cb;               // [M][ldcb] or null
    int64_t ldcb;
    int32_t relu;
};

constexpr int kGT = 64;      // tile edge
constexpr int kGK = 64;      // k step (two 32-wide chunks per operand)
constexpr int kGPad = 8;     // LDS row padding (bf16)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One thread's 8-element chunk of a 64 x 32 operand tile.  KC: row t/4,
// k offset 8 (t % 4); otherwise k row t/8, 8 consecutive m at 8 (t % 8).
// VEC: every chunk lies wholly inside or wholly outside the operand (16-byte
// aligned base, ld, K (KC) or rows (otherwise) multiples of 8 and at least
// 8), so a chunk is one unconditional 16-byte load from a clamped address
// and a mask (an AND, which the compiler does not turn back into a branch
// around the load): the compiler can then count the loads and keep those of
// later steps in flight.
template <bool KC, bool VEC>
struct Chunk {
    u32x4 v;

    __device__ __forceinline__ void load(const __bf16 *X, int64_t ld, int rows, int K, int r0,
                                         int k0)
    {
        const int t = threadIdx.x;
        union {
            u32x4 u;
            __bf16 h[8];
        } c;
        if (KC) {
            const int r = t >> 2, kk = (t & 3) * 8;
            const int gr = r0 + r, gk = k0 + kk;
            const __bf16 *p = X + (int64_t)gr * ld + gk;
            if (VEC) {
                // an unconditional load from a valid (clamped) address, then a select
                const u32x4 x = *reinterpret_cast<const u32x4 *>(X + (int64_t)min(gr, rows - 1) * ld +
                                                                 min(gk, K - 8));
                const uint32_t keep = (gr < rows && gk < K) ? 0xFFFFFFFFu : 0u;
                c.u = x & keep;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) c.h[e] = (gr < rows && gk + e < K) ? p[e] : (__bf16)0.0f;
            }
        } else {
            const int kk = t >> 3, rr = (t & 7) * 8;
            const int gk = k0 + kk, gr = r0 + rr;
            const __bf16 *p = X + (int64_t)gk * ld + gr;
            if (VEC) {
                const u32x4 x = *reinterpret_cast<const u32x4 *>(X + (int64_t)min(gk, K - 1) * ld +
                                                                 min(gr, rows - 8));
                const uint32_t keep = (gk < K && gr < rows) ? 0xFFFFFFFFu : 0u;
                c.u = x & keep;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) c.h[e] = (gk < K && gr + e < rows) ? p[e] : (__bf16)0.0f;
            }
        }
        v = c.u;
    }

    // into columns koff .. koff + 31 of the tile
    __device__ __forceinline__ void store(__bf16 (*S)[kGK + kGPad], int koff) const
    {
        const int t = threadIdx.x;
        if (KC) {
            *reinterpret_cast<u32x4 *>(&S[t >> 2][koff + (t & 3) * 8]) = v;
        } else {
            union {
                u32x4 u;
                __bf16 h[8];
            } c;
            c.u = v;
            const int kk = t >> 3, rr = (t & 7) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e) S[rr + e][koff + kk] = c.h[e];
        }
    }
};

// The K range is walked in steps of kGK = 64 (two 32-wide chunks per
// operand).  Each thread holds the chunks of the next ST steps in registers
// (a ring, refilled as each step is stored), so ST steps of loads are in
// flight behind the MFMAs (ST = 4 for long K; 1 keeps the registers, and the
// workgroups per CU, of short-K products); the LDS tiles are double-buffered,
// so one barrier per step suffices: a thread that stores step t + 1 into the
// buffer of step t - 1 has passed barrier t, which every thread reaches only
// after its MFMAs of step t - 1.
template <bool A_KC, bool B_KC, bool VEC, int ST>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) __bf16 sA[2][kGT][kGK + kGPad];
    __shared__ __attribute__((aligned(16))) __bf16 sB[2][kGT][kGK + kGPad];
    const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kb = blockIdx.z * g.kslice;
    const int ke = min(g.K, kb + g.kslice);
    f32x4m acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4m){0.f, 0.f, 0.f, 0.f};

    // chunks past ke or K are zero-filled by the loads; the steps are padded
    // to whole rounds of ST (the padding multiplies zeros), so the stage
    // loop has no exit and the accumulators stay in place
    Chunk<A_KC, VEC> ca[ST][2];
    Chunk<B_KC, VEC> cb[ST][2];
    const int nround = (ke - kb + ST * kGK - 1) / (ST * kGK);
    static_assert(ST == 1 || ST % 2 == 0, "the LDS buffer of a step is its parity");
#pragma unroll
    for (int st = 0; st < ST; ++st) {
        const int k0 = kb + st * kGK;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            ca[st][h].load(g.A, g.lda, g.M, ke, m0, k0 + 32 * h);
            cb[st][h].load(g.B, g.ldb, g.N, ke, n0, k0 + 32 * h);
        }
    }
    const int rl = lane & 15;
    for (int rd = 0; rd < nround; ++rd) {
#pragma unroll
        for (int st = 0; st < ST; ++st) {
            const int bf = ST == 1 ? (rd & 1) : (st & 1);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                ca[st][h].store(sA[bf], 32 * h);
                cb[st][h].store(sB[bf], 32 * h);
            }
            __syncthreads();
            // the chunks of the step ST later (zero past the end)
            const int kn = kb + ((rd + 1) * ST + st) * kGK;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                ca[st][h].load(g.A, g.lda, g.M, ke, m0, kn + 32 * h);
                cb[st][h].load(g.B, g.ldb, g.N, ke, n0, kn + 32 * h);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int kq = 32 * h + (lane >> 4) * 8;
                bf16x8 a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    a[i] = *reinterpret_cast<const bf16x8 *>(&sA[bf][wm + 16 * i + rl][kq]);
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    b[j] = *reinterpret_cast<const bf16x8 *>(&sB[bf][wn + 16 * j + rl][kq]);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
    }
    // D layout: lane holds rows 4*(lane/16) + r, column lane % 16 of each 16 x 16 block.
    const bool split = gridDim.z > 1;
    float *C = split ? g.C + (int64_t)blockIdx.z * g.M * g.ldc : g.C;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (split) {
                    C[(int64_t)m * g.ldc + n] = v;
                    continue;
                }
                if (g.bias) v += g.bias[n];
                if (g.relu) v = v > 0.f ? v : 0.f;
                if (g.mask && !((float)g.mask[(int64_t)m * g.ldm + n] > 0.f)) v = 0.f;
                if (g.C) C[(int64_t)m * g.ldc + n] = v;
                if (g.Cb) g.Cb[(int64_t)m * g.ldcb + n] = (__bf16)v;
            }
}

// Sum of the split-K partial products in slice order (deterministic):
// C[m][n] = sum_z part[z][m][n].
__global__ void k_splitk_sum(const float *part, int32_t S, int32_t M, int32_t N, int64_t ldc,
                             float *C)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)M * N) return;
    const int64_t m = idx / N, n = idx - m * N;
    float v = 0.0f;
    for (int z = 0; z < S; ++z) v += part[(int64_t)z * M * ldc + m * ldc + n];
    C[m * ldc + n] = v;
}

static bool vec_ok(const void *p, int64_t ld)
{
    return ((uintptr_t)p % 16) == 0 && (ld % 8) == 0;
}

template <bool A_KC, bool B_KC>
static void launch_gemm_kc(const GemmArgs &g, bool vec, bool deep, dim3 grid, hipStream_t s)
{
    if (vec && deep) hipLaunchKernelGGL((k_gemm<A_KC, B_KC, true, 4>), grid, dim3(256), 0, s, g);
    else if (vec) hipLaunchKernelGGL((k_gemm<A_KC, B_KC, true, 1>), grid, dim3(256), 0, s, g);
    else if (deep) hipLaunchKernelGGL((k_gemm<A_KC, B_KC, false, 4>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_gemm<A_KC, B_KC, false, 1>), grid, dim3(256), 0, s, g);
}

static void launch_gemm(const GemmArgs &g, bool a_kc, bool b_kc, bool vec, bool deep, dim3 grid,
                        hipStream_t s)
{
    if (a_kc && b_kc) launch_gemm_kc<true, true>(g, vec, deep, grid, s);
    else if (a_kc) launch_gemm_kc<true, false>(g, vec, deep, grid, s);
    else if (b_kc) launch_gemm_kc<false, true>(g, vec, deep, grid, s);
    else launch_gemm_kc<false, false>(g, vec, deep, grid, s);
}

// part: scratch for split-K partials (S * M * ldc floats) or null (no split).
static int gemm(GemmArgs g, bool a_kc, bool b_kc, hipStream_t s, arsel_ctx *ctx = nullptr,
                float *part = nullptr, size_t part_floats = 0)
{
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return ARSEL_OK;
    g.vec_a = vec_ok(g.A, g.lda);
    g.vec_b = vec_ok(g.B, g.ldb);
    dim3 grid((g.N + kGT - 1) / kGT, (g.M + kGT - 1) / kGT, 1);
    g.kslice = g.K;
    const bool plain = !g.bias && !g.relu && !g.mask && !g.Cb && g.C;
    float *C_final = g.C;
    int S = 1;
    if (ctx && part && plain && g.K >= 256) {
        const int tiles = (int)(grid.x * grid.y);
        while (S < 8 && tiles * S * 2 <= 2 * ctx->num_cu && g.K / (S * 2) >= 128 &&
               (size_t)(S * 2) * g.M * g.ldc <= part_floats)
            S *= 2;
    }
    if (S > 1) {
        g.kslice = ((g.K + S - 1) / S + kGK - 1) / kGK * kGK;
        S = (g.K + g.kslice - 1) / g.kslice;
        grid.z = S;
        g.C = part;
    }
    // whole-chunk operands (see Chunk): the K range of every split-K slice
    // is a multiple of the k step, so K itself decides
    const bool vec = g.vec_a && g.vec_b && g.K % 8 == 0 && (a_kc || g.M % 8 == 0) &&
                     (b_kc || g.N % 8 == 0);
    const bool deep = g.kslice >= 8 * kGK;   // at least two rounds of four steps
    launch_gemm(g, a_kc, b_kc, vec, deep, grid, s);
    if (S > 1) {
        const int64_t n = (int64_t)g.M * g.N;
        hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, S,
                           g.M, g.N, g.ldc, C_final);
    }
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

static GemmArgs gemm_args(const void *A, int64_t lda, const void *B, int64_t ldb, int M, int N, int K)
{
    GemmArgs g{};
    g.A = (const __bf16 *)A;
    g.B = (const __bf16 *)B;
    g.lda = lda;
    g.ldb = ldb;
    g.M = M;
    g.N = N;
    g.K = K;
    return g;
}

// ---------------------------------------------------------------------------
// Elementwise and row kernels.
// ---------------------------------------------------------------------------

// F[r][i] = bf16(log1p(X[r][i])) for i < N, 0 for N <= i < Kp.  Counts are
// integers, so 1 + x is exact in FP32 (x < 2^24) and the hardware logarithm
// (a few ulp) is far inside the BF16 rounding that follows.  Columns across
// the x dimension, rows strided over the y dimension.
__global__ void k_features(const int32_t *X, int32_t R, int32_t N, int32_t Kp, __bf16 *F)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Kp) return;
    for (int64_t r = blockIdx.y; r < R; r += gridDim.y) {
        float v = 0.0f;
        if (i < N) {
            const int32_t x = X[r * N + i];
            v = x > 0 ? __logf(1.0f + (float)x) : 0.0f;
        }
        F[r * Kp + i] = (__bf16)v;
    }
}

// One wavefront per row: masked softmax of z over alpha_j > 0, then Q.
// For training (dz_b / dz_f not null): dz_j = (q_j - p_j) * scale with
// p_j = alpha_j / sum alpha (FP32), written as BF16 and FP32; the row's
// cross-entropy -sum p_j log q_j goes to *ce_out (the kernel adds the
// workgroup's rows to the loss, scaled).  Rows of up to 64 * PER elements
// are read once into registers (one exp per element); longer rows loop over
// global memory (PER = 0).
__device__ __forceinline__ float wave_sum_f32(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ float wave_max_f32(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
    return x;
}

template <int PER>
__device__ void softmax_row(const float *z, const float *a, int64_t r, int32_t M, int32_t L,
                            float *q_out, uint32_t *Q_out, __bf16 *dz_b, float *dz_f,
                            int64_t lddz, float scale, float *ce_out, int lane)
{
    constexpr int NR = PER > 0 ? PER : 1;
    float zr[NR], ar[NR];
    auto zat = [&](int k, int j) { return PER > 0 ? zr[k] : z[j]; };
    auto aat = [&](int k, int j) { return PER > 0 ? ar[k] : a[j]; };
    const int iters = PER > 0 ? PER : (M + 63) / 64;
    float zmax = -INFINITY, asum = 0.0f;
#pragma unroll
    for (int k = 0; k < (PER > 0 ? PER : 1); ++k) {
        if (PER > 0) {
            const int j = lane + 64 * k;
            zr[k] = j < M ? z[j] : 0.0f;
            ar[k] = j < M ? a[j] : 0.0f;
        }
    }
    for (int k = 0; k < iters; ++k) {
        const int j = lane + 64 * k;
        if (j < M && aat(k, j) > 0.0f) {
            zmax = fmaxf(zmax, zat(k, j));
            asum += aat(k, j);
        }
    }
    zmax = wave_max_f32(zmax);
    asum = wave_sum_f32(asum);
    float esum = 0.0f;
    for (int k = 0; k < iters; ++k) {
        const int j = lane + 64 * k;
        const float e = (j < M && aat(k, j) > 0.0f) ? expf(zat(k, j) - zmax) : 0.0f;
        if (PER > 0) zr[k] = e;            // the row's exponentials replace its logits
        esum += e;
    }
    esum = wave_sum_f32(esum);
    const float qscale = ldexpf(1.0f, 31 - L);
    const float lse = zmax + logf(esum);
    float ce = 0.0f;
    for (int k = 0; k < iters; ++k) {
        const int j = lane + 64 * k;
        if (j >= M) break;
        const bool sup = aat(k, j) > 0.0f;
        const float e = PER > 0 ? zr[k] : (sup ? expf(z[j] - zmax) : 0.0f);
        const float q = sup ? e / esum : 0.0f;
        if (q_out) q_out[r * M + j] = q;
        if (Q_out) {
            uint32_t Q = 0;
            if (sup) {
                const float f = floorf(q * qscale);
                Q = f < 1.0f ? 1u : (uint32_t)f;
            }
            Q_out[r * M + j] = Q;
        }
        if (dz_b || dz_f) {
            const float p = sup ? aat(k, j) / asum : 0.0f;
            const float d = (q - p) * scale;
            if (dz_b) dz_b[r * lddz + j] = (__bf16)d;
            if (dz_f) dz_f[r * lddz + j] = d;
            if (sup && p > 0.0f) ce -= p * (z[j] - lse);
        }
    }
    // padded logits (M <= j < lddz) carry no gradient
    for (int j = M + lane; j < lddz; j += 64) {
        if (dz_b) dz_b[r * lddz + j] = (__bf16)0.0f;
        if (dz_f) dz_f[r * lddz + j] = 0.0f;
    }
    if (ce_out) {
        ce = wave_sum_f32(ce);
        if (lane == 0) *ce_out = ce;
    }
}

constexpr int kSoftmaxWaves = 16;   // rows (wavefronts) per workgroup
constexpr int kSoftmaxPer = 24;     // register-resident elements per lane (rows up to 1536)

__global__ __launch_bounds__(kSoftmaxWaves * 64) void k_softmax_quant(
    const float *Z, int64_t ldz, const float *alpha, int32_t R, int32_t M, int32_t L, float *q_out,
    uint32_t *Q_out, __bf16 *dz_b, float *dz_f, int64_t lddz, float scale, float *loss)
{
    __shared__ float ce_row[kSoftmaxWaves];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * kSoftmaxWaves + wave;
    if (r < R) {
        float *ce = loss ? &ce_row[wave] : nullptr;
        if (M <= 64 * 17)           // M = 1029 and below: 17 elements per lane
            softmax_row<17>(Z + r * ldz, alpha + r * M, r, M, L, q_out, Q_out, dz_b, dz_f, lddz,
                            scale, ce, lane);
        else if (M <= 64 * kSoftmaxPer)
            softmax_row<kSoftmaxPer>(Z + r * ldz, alpha + r * M, r, M, L, q_out, Q_out, dz_b,
                                     dz_f, lddz, scale, ce, lane);
        else
            softmax_row<0>(Z + r * ldz, alpha + r * M, r, M, L, q_out, Q_out, dz_b, dz_f, lddz,
                           scale, ce, lane);
    }
    else if (loss && lane == 0)
        ce_row[wave] = 0.0f;
    if (loss) {
        // the workgroup's rows summed in a fixed order, one atomic per workgroup
        // (one per row put 10^3 same-address atomics in series per training step)
        __syncthreads();
        if (threadIdx.x == 0) {
            float acc = 0.0f;
            for (int w = 0; w < kSoftmaxWaves; ++w) acc += ce_row[w];
            atomicAdd(loss, acc * scale);
        }
    }
}


// Column sums of a [R][ld] FP32 matrix (bias gradients): out[n] = sum_r D[r][n].
// A workgroup owns 64 columns; its 16 row groups each sum rows g, g+16, ...
// with four interleaved accumulators, then the partials are added in a fixed
// order, so the result does not depend on scheduling.
__global__ __launch_bounds__(1024) void k_colsum(const float *D, int64_t ld, int32_t R, int32_t N,
                                                 float *out)
{
    __shared__ float part[16][65];
    const int c = threadIdx.x & 63;
    const int g = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (n < N) {
        int r = g;
        for (; r + 48 < R; r += 64) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += D[(int64_t)(r + 16 * u) * ld + n];
        }
        for (int u = 0; r < R; r += 16, ++u) acc[u & 3] += D[(int64_t)r * ld + n];
    }
    part[g][c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (g == 0 && n < N) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) s += part[i][c];
        out[n] = s;
    }
}

// Adam on FP32 master weights (Kingma & Ba 2015, Algorithm 1: moments, bias
// corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t, update), refreshing the
// BF16 copy.  Every operation is a separately rounded FP32 operation in the
// order of the algorithm's update rules (no contraction; division and
// square root correctly rounded).
__global__ void k_adam(float *w, const float *g, float *m, float *v, __bf16 *wb, int64_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = (__bf16)wi;
}

__global__ void k_zero_f32(float *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

static inline dim3 grid1(int64_t n, int b = 256)
{
    return dim3((unsigned)((n + b - 1) / b));
}

// Workspace carved from one context-owned buffer.
struct Carver {
    char *base;
    size_t off;
    template <class T>
    T *take(size_t n)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = (T *)(base + off);
        off += n * sizeof(T);
        return p;
    }
};

static int ensure_ws(arsel_ctx *ctx, size_t bytes)
{
    return ctx_grow(ctx, &ctx->ws, &ctx->ws_bytes, bytes);
}

static int check_mlp(const arsel_mlp *n)
{
    if (!n || !n->W1 || !n->W2 || !n->W3 || !n->b1 || !n->b2 || !n->b3) return ARSEL_ERR_NULL;
    if (n->N < 1 || n->M < 1 || n->H < 1 || n->Kp < n->N || n->Mp < n->M) return ARSEL_ERR_SIZE;
    return ARSEL_OK;
}

static int ceil_log2_host(int32_t m)
{
    int L = 0;
    while ((1ll << L) < m) ++L;
    return L;
}

// Forward pass into the workspace; returns pointers to F, H1, H2, Z.
struct Fwd {
    __bf16 *F, *H1, *H2;
    float *Z;
};

static int forward(arsel_ctx *ctx, const arsel_mlp *n, const int32_t *X, int32_t R, Carver &cv,
                   Fwd &f, hipStream_t s)
{
    f.F = cv.take<__bf16>((size_t)R * n->Kp);
    f.H1 = cv.take<__bf16>((size_t)R * n->H);
    f.H2 = cv.take<__bf16>((size_t)R * n->H);
    f.Z = cv.take<float>((size_t)R * n->Mp);
    (void)ctx;
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n->Kp + 255) / 256), (unsigned)std::min(R, 65535)),
                       dim3(256), 0, s, X, R, n->N, n->Kp, f.F);
    GemmArgs g = gemm_args(f.F, n->Kp, n->W1, n->Kp, R, n->H, n->Kp);
    g.bias = n->b1;
    g.relu = 1;
    g.Cb = f.H1;
    g.ldcb = n->H;
    int rc = gemm(g, true, true, s);
    if (rc) return rc;
    g = gemm_args(f.H1, n->H, n->W2, n->H, R, n->H, n->H);
    g.bias = n->b2;
    g.relu = 1;
    g.Cb = f.H2;
    g.ldcb = n->H;
    if ((rc = gemm(g, true, true, s))) return rc;
    g = gemm_args(f.H2, n->H, n->W3, n->H, R, n->Mp, n->H);
    g.bias = n->b3;
    g.C = f.Z;
    g.ldc = n->Mp;
    return gemm(g, true, true, s);
}

// ---------------------------------------------------------------------------
// Fused inference forward: one workgroup of kFW wavefronts per block of kFB
// states runs the features, the three layers, the masked softmax and the
// quantisation; f, h1 and h2 stay in LDS, z stays in the MFMA accumulators,
// and the weights stream from L2 straight into MFMA operand registers.  The
// k order of every product is the layer-by-layer kernels' (32-wide chunks in
// increasing k) and the epilogues are theirs, so f, h1, h2, z and the
// exponentials are bit-identical to the unfused path; only the softmax row
// sums are added in another order.  Shapes: H = 256, Kp % 32 == 0 and
// Kp <= kFMaxKp, Mp % 16 == 0 and Mp <= 16 * kFW * kFT3; others take the
// unfused path.
// ---------------------------------------------------------------------------
constexpr int kFB = 32;            // states per workgroup (two 16-row MFMA tiles)
constexpr int kFW = 8;             // wavefronts per workgroup
constexpr int kFH = 256;           // hidden width
constexpr int kFT3 = 10;           // layer-3 column tiles per wavefront (Mp <= 1280)
constexpr int kFMaxKp = 1024;
constexpr int kFPad = 8;           // LDS row padding (bf16)

struct FusedFwd {
    const int32_t *X;
    const float *alpha;
    const __bf16 *W1, *W2, *W3;
    const float *b1, *b2, *b3;
    float *q_out;
    uint32_t *Q_out;
    int32_t R, N, M, Kp, Mp, L;
};

__device__ __forceinline__ bf16x8 ld_frag(const __bf16 *p)
{
    return *reinterpret_cast<const bf16x8 *>(p);
}

// Max over the 16 lanes of each DPP row (rotations: every lane gets it).
__device__ __forceinline__ float row16_max(float x)
{
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xF, 0xF, false)));
    x = fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false)));
    return x;
}

// Inclusive sum over the 16 lanes of each DPP row; lane 15 of a row holds
// the row's total (lanes without a source add 0).
__device__ __forceinline__ float row16_sum_to_last(float x)
{
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x112, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xF, 0xF, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xF, 0xF, false));
    return x;
}

// One hidden layer of the fused forward: dst[m][n] = bf16(relu(sum_k
// src[m][k] W[n][k] + b[n])) for the block's 32 rows and 256 outputs; wave w
// owns columns 32 w .. 32 w + 31.
__device__ __forceinline__ void fused_hidden(const __bf16 *src, int lds_src, const __bf16 *W,
                                             int K, const float *bias, __bf16 *dst, int lds_dst)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rl = lane & 15, kq = (lane >> 4) * 8;
    f32x4m acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[i][c] = (f32x4m){0.f, 0.f, 0.f, 0.f};
    const __bf16 *wrow[2] = {W + (int64_t)(32 * wave + rl) * K + kq,
                             W + (int64_t)(32 * wave + 16 + rl) * K + kq};
    bf16x8 b[2], bn[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) b[c] = ld_frag(wrow[c]);
    for (int k0 = 0; k0 < K; k0 += 32) {
        if (k0 + 32 < K) {
#pragma unroll
            for (int c = 0; c < 2; ++c) bn[c] = ld_frag(wrow[c] + k0 + 32);
        }
        bf16x8 a[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = ld_frag(src + (16 * i + rl) * lds_src + k0 + kq);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                acc[i][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[c], acc[i][c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < 2; ++c) b[c] = bn[c];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int n = 32 * wave + 16 * c + rl;
        const float bb = bias[n];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[i][c][r] + bb;
                v = v > 0.f ? v : 0.f;
                dst[(16 * i + 4 * (lane >> 4) + r) * lds_dst + n] = (__bf16)v;
            }
    }
}

__global__ __launch_bounds__(kFW * 64) void k_mlp_forward_fused(FusedFwd f)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char fsm[];
    const int ldf = f.Kp + kFPad, ldh = kFH + kFPad;
    __bf16 *sF = reinterpret_cast<__bf16 *>(fsm);                    // [32][Kp + 8], later h2
    __bf16 *sH1 = sF + kFB * ldf;                                     // [32][264]
    float *sRed = reinterpret_cast<float *>(sH1 + kFB * ldh);         // [kFW][32]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rl = lane & 15, kq = (lane >> 4) * 8;
    const int64_t r0 = (int64_t)blockIdx.x * kFB;

    // features: bf16(log1p(x)) as the unfused feature kernel computes them
    for (int e = tid; e < kFB * f.Kp; e += kFW * 64) {
        const int m = e / f.Kp, i = e - m * f.Kp;
        const int64_t r = r0 + m;
        float v = 0.0f;
        if (i < f.N && r < f.R) {
            const int32_t x = f.X[r * f.N + i];
            v = x > 0 ? __logf(1.0f + (float)x) : 0.0f;
        }
        sF[m * ldf + i] = (__bf16)v;
    }
    __syncthreads();
    fused_hidden(sF, ldf, f.W1, f.Kp, f.b1, sH1, ldh);
    __syncthreads();
    __bf16 *sH2 = sF;
    fused_hidden(sH1, ldh, f.W2, kFH, f.b2, sH2, ldh);
    __syncthreads();

    // layer 3: wave w owns column tiles w, w + kFW, ... (z in registers)
    const int ntiles = f.Mp >> 4;
    f32x4m acc[2][kFT3];
#pragma unroll
    for (int t = 0; t < kFT3; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[i][t] = (f32x4m){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < kFH; k0 += 32) {
        bf16x8 a[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = ld_frag(sH2 + (16 * i + rl) * ldh + k0 + kq);
#pragma unroll
        for (int t = 0; t < kFT3; ++t) {
            const int tile = wave + kFW * t;
            if (tile < ntiles) {
                const bf16x8 b = ld_frag(f.W3 + (int64_t)(16 * tile + rl) * kFH + k0 + kq);
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b, acc[i][t], 0, 0, 0);
            }
        }
    }

    // masked softmax over alpha_j > 0 and quantisation.  Lane (i, r) rows:
    // m = 16 i + 4 (lane / 16) + r; column of tile t: n = 16 tile + lane % 16.
    uint32_t sup[kFT3];
    float rmax[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) rmax[i][r] = -INFINITY;
#pragma unroll
    for (int t = 0; t < kFT3; ++t) {
        sup[t] = 0;
        const int tile = wave + kFW * t;
        const int n = 16 * tile + rl;
        const float bb = (tile < ntiles) ? f.b3[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + 16 * i + 4 * (lane >> 4) + r;
                const float z = acc[i][t][r] + bb;
                acc[i][t][r] = z;
                if (tile < ntiles && n < f.M && row < f.R && f.alpha[row * f.M + n] > 0.0f) {
                    sup[t] |= 1u << (4 * i + r);
                    rmax[i][r] = fmaxf(rmax[i][r], z);
                }
            }
    }
    // row maxima: the 16 lanes of a DPP row, then the waves through LDS
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float x = row16_max(rmax[i][r]);
            if (rl == 15) sRed[wave * kFB + 16 * i + 4 * (lane >> 4) + r] = x;
        }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * i + 4 * (lane >> 4) + r;
            float x = -INFINITY;
            for (int w = 0; w < kFW; ++w) x = fmaxf(x, sRed[w * kFB + m]);
            rmax[i][r] = x;
        }
    __syncthreads();
    // exponentials (replacing z) and their row sums
    float rsum[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) rsum[i][r] = 0.0f;
#pragma unroll
    for (int t = 0; t < kFT3; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float e = (sup[t] >> (4 * i + r)) & 1u ? expf(acc[i][t][r] - rmax[i][r]) : 0.0f;
                acc[i][t][r] = e;
                rsum[i][r] += e;
            }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float x = row16_sum_to_last(rsum[i][r]);
            if (rl == 15) sRed[wave * kFB + 16 * i + 4 * (lane >> 4) + r] = x;
        }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * i + 4 * (lane >> 4) + r;
            float x = 0.0f;
            for (int w = 0; w < kFW; ++w) x += sRed[w * kFB + m];
            rsum[i][r] = x;
        }
    const float qscale = ldexpf(1.0f, 31 - f.L);
#pragma unroll
    for (int t = 0; t < kFT3; ++t) {
        const int tile = wave + kFW * t;
        const int n = 16 * tile + rl;
        if (tile >= ntiles || n >= f.M) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = r0 + 16 * i + 4 * (lane >> 4) + r;
                if (row >= f.R) continue;
                const bool s = (sup[t] >> (4 * i + r)) & 1u;
                const float q = s ? acc[i][t][r] / rsum[i][r] : 0.0f;
                if (f.q_out) f.q_out[row * f.M + n] = q;
                if (f.Q_out) {
                    uint32_t Q = 0;
                    if (s) {
                        const float fl = floorf(q * qscale);
                        Q = fl < 1.0f ? 1u : (uint32_t)fl;
                    }
                    f.Q_out[row * f.M + n] = Q;
                }
            }
    }
}

static size_t fused_lds_bytes(int32_t Kp)
{
    return (size_t)kFB * (Kp + kFPad) * 2 + (size_t)kFB * (kFH + kFPad) * 2 + (size_t)kFW * kFB * 4;
}

static bool fused_ok(arsel_ctx *ctx, const arsel_mlp *n)
{
    const auto al = [](const void *p) { return ((uintptr_t)p % 16) == 0; };
    return ctx->mlp_fused && n->H == kFH && n->Kp % 32 == 0 && n->Kp <= kFMaxKp &&
           n->Mp % 16 == 0 && n->Mp <= 16 * kFW * kFT3 && al(n->W1) && al(n->W2) && al(n->W3) &&
           fused_lds_bytes(n->Kp) <= ctx->lds_per_block;
}

static size_t fwd_bytes(const arsel_mlp *n, int32_t R)
{
    return (size_t)R * (n->Kp * 2 + n->H * 4 + n->Mp * 4) + 8 * 256;
}

}  // namespace arsel

using namespace arsel;

extern "C" int arsel_mlp_forward(arsel_ctx *ctx, const arsel_mlp *net, const int32_t *X, int32_t R,
                                 const float *alpha, float *q_out, uint32_t *Q_out, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    int rc = check_mlp(net);
    if (rc) return rc;
    if (R < 0) return ARSEL_ERR_SIZE;
    if (R == 0) return ARSEL_OK;
    if (!X || !alpha || (!q_out && !Q_out)) return ARSEL_ERR_NULL;
    if ((rc = ctx_activate(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (fused_ok(ctx, net)) {
        FusedFwd f;
        f.X = X;
        f.alpha = alpha;
        f.W1 = (const __bf16 *)net->W1;
        f.W2 = (const __bf16 *)net->W2;
        f.W3 = (const __bf16 *)net->W3;
        f.b1 = net->b1;
        f.b2 = net->b2;
        f.b3 = net->b3;
        f.q_out = q_out;
        f.Q_out = Q_out;
        f.R = R;
        f.N = net->N;
        f.M = net->M;
        f.Kp = net->Kp;
        f.Mp = net->Mp;
        f.L = ceil_log2_host(net->M);
        hipLaunchKernelGGL(k_mlp_forward_fused, dim3((R + kFB - 1) / kFB), dim3(kFW * 64),
                           fused_lds_bytes(net->Kp), s, f);
        return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
    }
    if ((rc = ensure_ws(ctx, fwd_bytes(net, R)))) return rc;
    Carver cv{(char *)ctx->ws, 0};
    Fwd f;
    if ((rc = forward(ctx, net, X, R, cv, f, s))) return rc;
    hipLaunchKernelGGL(k_softmax_quant, dim3((R + kSoftmaxWaves - 1) / kSoftmaxWaves),
                       dim3(kSoftmaxWaves * 64), 0, s, f.Z, (int64_t)net->Mp,
                       alpha, R, net->M, ceil_log2_host(net->M), q_out, Q_out, (__bf16 *)nullptr,
                       (float *)nullptr, (int64_t)0, 0.0f, (float *)nullptr);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

extern "C" int arsel_mlp_train_step(arsel_ctx *ctx, const arsel_mlp_train *tr, const int32_t *X,
                                    const float *alpha, int32_t B, float lr, int32_t t,
                                    float *loss, void *stream)
{
    if (!ctx || !tr) return ARSEL_ERR_NULL;
    const arsel_mlp *n = &tr->net;
    int rc = check_mlp(n);
    if (rc) return rc;
    if (B < 1 || t < 1) return ARSEL_ERR_SIZE;
    if (!X || !alpha || !loss) return ARSEL_ERR_NULL;
    for (int i = 0; i < 6; ++i)
        if (!tr->master[i] || !tr->grad[i] || !tr->m[i] || !tr->v[i]) return ARSEL_ERR_NULL;
    if ((rc = ctx_activate(ctx))) return rc;
    const size_t extra = (size_t)B * (n->Mp * 6 + n->H * 12) + 8 * 256 +
                         (size_t)8 * std::max<size_t>((size_t)n->Mp * n->H, (size_t)n->H * n->Kp) * 4 + 256;
    if ((rc = ensure_ws(ctx, fwd_bytes(n, B) + extra))) return rc;
    hipStream_t s = (hipStream_t)stream;
    Carver cv{(char *)ctx->ws, 0};
    Fwd f;
    if ((rc = forward(ctx, n, X, B, cv, f, s))) return rc;
    __bf16 *dZb = cv.take<__bf16>((size_t)B * n->Mp);
    float *dZf = cv.take<float>((size_t)B * n->Mp);
    __bf16 *dH2 = cv.take<__bf16>((size_t)B * n->H);
    float *dH2f = cv.take<float>((size_t)B * n->H);
    __bf16 *dH1 = cv.take<__bf16>((size_t)B * n->H);
    float *dH1f = cv.take<float>((size_t)B * n->H);
    const size_t part_n = (size_t)8 * std::max<size_t>((size_t)n->Mp * n->H, (size_t)n->H * n->Kp);
    float *part = cv.take<float>(part_n);

    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, s, loss, (int64_t)1);
    const float scale = 1.0f / (float)B;
    hipLaunchKernelGGL(k_softmax_quant, dim3((B + kSoftmaxWaves - 1) / kSoftmaxWaves),
                       dim3(kSoftmaxWaves * 64), 0, s, f.Z, (int64_t)n->Mp, alpha,
                       B, n->M, ceil_log2_host(n->M), (float *)nullptr, (uint32_t *)nullptr, dZb, dZf,
                       (int64_t)n->Mp, scale, loss);
    // gradients: grad[0..5] = dW1, db1, dW2, db2, dW3, db3 (FP32, shapes of the masters)
    GemmArgs g = gemm_args(dZb, n->Mp, f.H2, n->H, n->Mp, n->H, B);     // dW3 = dZ^T H2
    g.C = tr->grad[4];
    g.ldc = n->H;
    if ((rc = gemm(g, false, false, s, ctx, part, part_n))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3((n->Mp + 63) / 64), dim3(1024), 0, s, dZf, (int64_t)n->Mp, B, n->Mp, tr->grad[5]);
    g = gemm_args(dZb, n->Mp, n->W3, n->H, B, n->H, n->Mp);              // dH2 = dZ W3 . [h2 > 0]
    g.mask = f.H2;
    g.ldm = n->H;
    g.Cb = dH2;
    g.ldcb = n->H;
    g.C = dH2f;
    g.ldc = n->H;
    if ((rc = gemm(g, true, false, s))) return rc;
    g = gemm_args(dH2, n->H, f.H1, n->H, n->H, n->H, B);                 // dW2 = dH2^T H1
    g.C = tr->grad[2];
    g.ldc = n->H;
    if ((rc = gemm(g, false, false, s, ctx, part, part_n))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3((n->H + 63) / 64), dim3(1024), 0, s, dH2f, (int64_t)n->H, B, n->H, tr->grad[3]);
    g = gemm_args(dH2, n->H, n->W2, n->H, B, n->H, n->H);                // dH1 = dH2 W2 . [h1 > 0]
    g.mask = f.H1;
    g.ldm = n->H;
    g.Cb = dH1;
    g.ldcb = n->H;
    g.C = dH1f;
    g.ldc = n->H;
    if ((rc = gemm(g, true, false, s))) return rc;
    g = gemm_args(dH1, n->H, f.F, n->Kp, n->H, n->Kp, B);                // dW1 = dH1^T F
    g.C = tr->grad[0];
    g.ldc = n->Kp;
    if ((rc = gemm(g, false, false, s, ctx, part, part_n))) return rc;
    hipLaunchKernelGGL(k_colsum, dim3((n->H + 63) / 64), dim3(1024), 0, s, dH1f, (int64_t)n->H, B, n->H, tr->grad[1]);

    const int64_t sizes[6] = {(int64_t)n->H * n->Kp, n->H, (int64_t)n->H * n->H, n->H,
                              (int64_t)n->Mp * n->H, n->Mp};
    __bf16 *copies[6] = {(__bf16 *)n->W1, nullptr, (__bf16 *)n->W2, nullptr, (__bf16 *)n->W3, nullptr};
    // bias corrections: binary64 power of the FP32 betas, rounded once to FP32
    const float c1 = (float)(1.0 - pow((double)tr->beta1, (double)t));
    const float c2 = (float)(1.0 - pow((double)tr->beta2, (double)t));
    for (int i = 0; i < 6; ++i)
        hipLaunchKernelGGL(k_adam, grid1(sizes[i]), dim3(256), 0, s, tr->master[i], tr->grad[i], tr->m[i],
                           tr->v[i], copies[i], sizes[i], lr, tr->beta1, tr->beta2, tr->eps, c1, c2);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

// Plain GEMM entry (tests and tools): C = A . B with the layout flags above.
extern "C" int arsel_gemm_bf16(arsel_ctx *ctx, const void *A, int64_t lda, int32_t a_kcontig,
                               const void *B, int64_t ldb, int32_t b_kcontig, int32_t M, int32_t N,
                               int32_t K, const float *bias, int32_t relu, float *C, int64_t ldc,
                               void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    if (M < 0 || N < 0 || K < 0) return ARSEL_ERR_SIZE;
    if (!A || !B || !C) return ARSEL_ERR_NULL;
    int rc = ctx_activate(ctx);
    if (rc) return rc;
    GemmArgs g = gemm_args(A, lda, B, ldb, M, N, K);
    g.bias = bias;
    g.relu = relu;
    g.C = C;
    g.ldc = ldc;
    return gemm(g, a_kcontig != 0, b_kcontig != 0, (hipStream_t)stream);
}

namespace arsel {
__global__ void k_cast_bf16(const float *w, __bf16 *wb, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = (__bf16)w[i];
}
}  // namespace arsel

// Refresh the BF16 copies W1, W2, W3 of a training state from its FP32 masters.
extern "C" int arsel_mlp_sync_bf16(arsel_ctx *ctx, const arsel_mlp_train *tr, void *stream)
{
    if (!ctx || !tr) return ARSEL_ERR_NULL;
    const arsel_mlp *n = &tr->net;
    int rc = check_mlp(n);
    if (rc) return rc;
    if (!tr->master[0] || !tr->master[2] || !tr->master[4]) return ARSEL_ERR_NULL;
    if ((rc = ctx_activate(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n1 = (int64_t)n->H * n->Kp, n2 = (int64_t)n->H * n->H, n3 = (int64_t)n->Mp * n->H;
    hipLaunchKernelGGL(k_cast_bf16, grid1(n1), dim3(256), 0, s, tr->master[0], (__bf16 *)n->W1, n1);
    hipLaunchKernelGGL(k_cast_bf16, grid1(n2), dim3(256), 0, s, tr->master[2], (__bf16 *)n->W2, n2);
    hipLaunchKernelGGL(k_cast_bf16, grid1(n3), dim3(256), 0, s, tr->master[4], (__bf16 *)n->W3, n3);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

// Forward path switch (tests compare the two; results are identical).
extern "C" int arsel_set_mlp_fused(arsel_ctx *ctx, int32_t on)
{
    if (!ctx) return ARSEL_ERR_NULL;
    ctx->mlp_fused = on != 0;
    return ARSEL_OK;
}
