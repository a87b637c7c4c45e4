// Workgroup-level pieces of the selection: reductions and scans over the
// NW wavefronts of a workgroup, and the staged loads of a row piece.
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

// Loads of one piece [p0, p0 + n) of a row, n = min(piece, M - p0) (piece a
// multiple of 4 floats, at most kStreamBatch float4 per thread of NT): an
// unaligned head of up to 3 elements, nq aligned float4 slots and a tail of
// up to 3, all issued before any is used.  Wavefront w holds the slots
// [w W, (w + 1) W), W = ceil(nq / NW) rounded up to 64, lane l of it the slots
// w W + 64 u + l (each load instruction reads 1 KB contiguous), so the piece
// splits into ordered wavefront ranges: wave 0 from element 0 (it holds the
// head), wave w from its first slot (or the tail's start when it has none),
// the last wave to the end (it holds the tail); a wave's part of the
// fixed-point sum is the sum over its range.  store() writes the piece to
// buf[0 .. n) and returns the thread's part of the sum.
template <int NT>
struct PieceLoads {
    static constexpr int NW = NT / kWave;
    f32x4 v[kStreamBatch];
    float hx, tx;

    struct Span {
        uint32_t n, head, nq, W;
    };

    __device__ __forceinline__ static Span span(const float *row, uint32_t M, uint32_t p0, uint32_t piece)
    {
        Span sp;
        sp.n = min(piece, M - p0);
        const uint32_t align = (uint32_t)(((16 - ((uintptr_t)(row + p0) & 15)) & 15) >> 2);
        sp.head = align < sp.n ? align : sp.n;
        sp.nq = (sp.n - sp.head) >> 2;
        sp.W = ((sp.nq + NW - 1) / NW + kWave - 1) / kWave * kWave;
        return sp;
    }

    // first element of wavefront w's range; wave w ends where wave w + 1
    // begins, the last wave at n
    __device__ __forceinline__ static uint32_t wave_begin(const Span &sp, uint32_t w)
    {
        return w == 0 ? 0u : sp.head + 4 * min(sp.W * w, sp.nq);
    }

    __device__ __forceinline__ void issue(const float *row, uint32_t M, uint32_t p0, uint32_t piece,
                                          uint32_t tid)
    {
        const Span sp = span(row, M, p0, piece);
        const float *s4 = row + p0 + sp.head;
        const uint32_t base = (tid >> 6) * sp.W + (tid & (kWave - 1));
        const uint32_t end = min((tid >> 6) * sp.W + sp.W, sp.nq);
#pragma unroll
        for (int u = 0; u < kStreamBatch; ++u) {
            const uint32_t i = base + u * kWave;
            if (i < end) v[u] = load_stream4(s4 + 4 * i);
        }
        hx = tid < sp.head ? row[p0 + tid] : 0.0f;
        const uint32_t t0 = sp.head + 4 * sp.nq, tl = tid - (NT - kWave);
        tx = tid >= NT - kWave && tl < sp.n - t0 ? row[p0 + t0 + tl] : 0.0f;
    }

    // LE39: every element's fixed-point exponent is at most 39 (see
    // fixed_weight_le39), true when the row's maximum is a normal float.
    template <bool LE39>
    __device__ __forceinline__ uint64_t store(const float *row, uint32_t M, uint32_t p0, uint32_t piece,
                                              uint32_t tid, float *buf, int shift) const
    {
        auto fw = [shift](float x) { return LE39 ? fixed_weight_le39(x, shift) : fixed_weight(x, shift); };
        const Span sp = span(row, M, p0, piece);
        const uint32_t base = (tid >> 6) * sp.W + (tid & (kWave - 1));
        const uint32_t end = min((tid >> 6) * sp.W + sp.W, sp.nq);
        uint64_t part = 0;
#pragma unroll
        for (int u = 0; u < kStreamBatch; ++u) {
            const uint32_t i = base + u * kWave;
            if (i < end) {
                float *d = buf + sp.head + 4 * i;
                d[0] = v[u].x;
                d[1] = v[u].y;
                d[2] = v[u].z;
                d[3] = v[u].w;
                part += fw(v[u].x) + fw(v[u].y);
                part += fw(v[u].z) + fw(v[u].w);
            }
            __builtin_amdgcn_sched_barrier(0);   // one slot's temporaries at a time
        }
        if (tid < sp.head) {
            buf[tid] = hx;
            part += fw(hx);
        }
        const uint32_t t0 = sp.head + 4 * sp.nq, tl = tid - (NT - kWave);
        if (tid >= NT - kWave && tl < sp.n - t0) {
            buf[t0 + tl] = tx;
            part += fw(tx);
        }
        return part;
    }
};

}  // namespace arsel
