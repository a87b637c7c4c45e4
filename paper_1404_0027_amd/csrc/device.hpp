// Device primitives for the acceptance-rejection selector on gfx950 (wave64).
//
// Philox4x32-10 (Salmon et al., SC'11), exactly-uniform candidate draws,
// wavefront reductions and scans, and the exact fixed-point arithmetic of
// the inverse-transform fallback.  Everything here is __device__ so that
// every kernel (dense, ragged, proposal, SSA) shares one definition.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace arsel {

constexpr int kWave = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// 16-byte streaming load (the data is read once and kept in LDS or registers).
__device__ __forceinline__ f32x4 load_stream4(const float *p)
{
    return __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
}

constexpr int kXcds = 8;         // MI355X: 8 XCDs, workgroups dealt round-robin

// Workgroups are dealt to the XCDs round-robin, so consecutive block ids land
// on different L2s.  Remap so that each XCD owns a contiguous range of tiles:
// the two halves of a 128-byte line of an SoA row then meet in one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int full = nb - nb % kXcds;
    if (b >= full) return b;
    return (b % kXcds) * (full / kXcds) + b / kXcds;
}

// ---------------------------------------------------------------------------
// Philox4x32-10: 10 rounds of two 32x32->64 multiplies; the key is bumped by
// the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct Words {
    uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c in one gfx950 three-input bitwise instruction (truth table 0x96);
// the compiler otherwise emits two two-input XORs.  Measured: a Philox block
// per wavefront drops from ~253 to ~175 SIMD cycles.
__device__ __forceinline__ uint32_t xor3_u32(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_u32((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3_u32((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

enum : uint32_t { kTagUniform = 0, kTagProposal = 1, kTagSSA = 2 };
constexpr uint32_t kFallbackBlock = 0xFFFFFFFFu;

// The fixed part of one instance's counter: (block, inst, step lo, step hi ^ tag<<28).
struct Stream {
    uint32_t k0, k1;   // key = seed
    uint32_t inst;
    uint32_t s_lo, s_hi;
    __device__ __forceinline__ Words block(uint32_t b) const
    {
        return philox4x32_10(b, inst, s_lo, s_hi, k0, k1);
    }
};

__device__ __forceinline__ Stream make_stream(uint64_t seed, uint64_t step, uint32_t inst,
                                              uint32_t tag)
{
    Stream s;
    s.k0 = (uint32_t)seed;
    s.k1 = (uint32_t)(seed >> 32);
    s.inst = inst;
    s.s_lo = (uint32_t)step;
    s.s_hi = (uint32_t)(step >> 32) ^ (tag << 28);
    return s;
}

// Lemire multiply-shift: candidate = hi32(w * n); the draw is rejected when
// lo32(w * n) < 2^32 mod n, which leaves exactly floor(2^32 / n) preimages
// per candidate.
__device__ __forceinline__ uint32_t lemire_threshold(uint32_t n)
{
    return (0u - n) % n;
}

__device__ __forceinline__ bool lemire(uint32_t w, uint32_t n, uint32_t thresh, uint32_t &j)
{
    const uint64_t m = (uint64_t)w * n;
    j = (uint32_t)(m >> 32);
    return (uint32_t)m >= thresh;
}

// u = w * 2^-32 exactly, as binary64.
__device__ __forceinline__ double grid_u(uint32_t w)
{
    return (double)w * 0x1p-32;
}

// ---------------------------------------------------------------------------
// Wavefront reductions (all 64 lanes active).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id()
{
    return (int)(threadIdx.x & (kWave - 1));
}

__device__ __forceinline__ float wave_max(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, kWave));
    return x;
}

// DPP move: lane receives src from the lane selected by CTRL; lanes with no
// source (or masked rows) receive 0, the identity of an unsigned maximum.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)src, CTRL, ROW_MASK, 0xF, false);
}

// Unsigned maximum over the 64 lanes with DPP row shifts and row broadcasts
// (no LDS traffic); every lane returns the result.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x)
{
    x = max(x, dpp_u32<0x111>(x));          // row_shr:1
    x = max(x, dpp_u32<0x112>(x));          // row_shr:2
    x = max(x, dpp_u32<0x114>(x));          // row_shr:4
    x = max(x, dpp_u32<0x118>(x));          // row_shr:8 -> lane 15 of each row: row max
    x = max(x, dpp_u32<0x142, 0xA>(x));     // row_bcast:15 into rows 1 and 3
    x = max(x, dpp_u32<0x143, 0xC>(x));     // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Inclusive prefix sum over the 64 lanes (u32, wrapping) with DPP: row
// shifts 1, 2, 4, 8 scan each row of 16 lanes, then row broadcasts carry the
// totals of rows 0..2 into the rows above.  No LDS traffic.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x)
{
    x += dpp_u32<0x111>(x);          // row_shr:1
    x += dpp_u32<0x112>(x);          // row_shr:2
    x += dpp_u32<0x114>(x);          // row_shr:4
    x += dpp_u32<0x118>(x);          // row_shr:8
    x += dpp_u32<0x142, 0xA>(x);     // row_bcast:15 into rows 1 and 3
    x += dpp_u32<0x143, 0xC>(x);     // row_bcast:31 into rows 2 and 3
    return x;
}

// Maximum over the lanes of the same row whose index is congruent mod 4:
// lane l returns max over lanes (l & ~15) + ((l + 4 i) & 15), i = 0..3.
__device__ __forceinline__ uint32_t row_max_mod4(uint32_t x)
{
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x124, 0xF, 0xF, false)); // row_ror:4
    x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x128, 0xF, 0xF, false)); // row_ror:8
    return x;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int off)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, off, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), off, kWave);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t x, int d)
{
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)x, d, kWave);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(x >> 32), d, kWave);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += shfl_xor_u64(x, off);
    return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = shfl_up_u64(x, d);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t x, int lane)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int lane)
{
    return (uint64_t)readlane_u32((uint32_t)x, lane) |
           ((uint64_t)readlane_u32((uint32_t)(x >> 32), lane) << 32);
}

// Wave-uniform copy of a value (held in a scalar register).  Loop and branch
// conditions of code that uses cross-lane operations are taken from such
// values, so that the compiler keeps the wave converged around them.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    return (uint64_t)uniform_u32((uint32_t)x) | ((uint64_t)uniform_u32((uint32_t)(x >> 32)) << 32);
}

// Fetch-and-add executed by the whole (converged) wave: lane 0 adds v, the
// other lanes add 0; every lane gets lane 0's old value, as a uniform value.
// Works on global and LDS addresses.
__device__ __forceinline__ uint32_t wave_fetch_add(uint32_t *p, uint32_t v)
{
    const uint32_t old = atomicAdd(p, (threadIdx.x & (kWave - 1)) == 0 ? v : 0u);
    return uniform_u32(old);
}

__device__ __forceinline__ int first_lane(uint64_t mask)
{
    return mask ? (int)__builtin_ctzll(mask) : kWave;
}

// ---------------------------------------------------------------------------
// Exact fixed point for the fallback.
// ---------------------------------------------------------------------------

// E with 2^(E-1) <= x < 2^E, for finite x > 0 (normal or subnormal).
__device__ __forceinline__ int exponent_above(float x)
{
    const uint32_t b = __float_as_uint(x);
    const uint32_t e = (b >> 23) & 0xFFu;
    if (e != 0) return (int)e - 126;
    const uint32_t m = b & 0x7FFFFFu;
    return (32 - __clz((int)m)) - 149;
}

// ceil(log2 n), 0 for n = 1.
__device__ __forceinline__ int ceil_log2_u32(uint32_t n)
{
    return n <= 1 ? 0 : 32 - __clz((int)(n - 1));
}

// floor(a * 2^shift) for a >= 0 finite, from the bits of a: a = m * 2^s' with
// m the 24-bit significand (implicit bit for normal numbers) and
// s' = max(e, 1) - 150.  The caller guarantees the result < 2^63.  Branch-free:
// with s = s' + shift, floor(m 2^s) is (m 2^39) >> (39 - s) for s <= 39 (the
// right shift drops the fraction; m < 2^24, so a shift of 63 already gives 0)
// and m << s above; both shift amounts are clamped to [0, 63].
__device__ __forceinline__ uint64_t fixed_weight(float a, int shift)
{
    const uint32_t b = __float_as_uint(a);
    const uint32_t e = (b >> 23) & 0xFFu;
    const uint32_t m = (b & 0x7FFFFFu) | (min(e, 1u) << 23);
    const int s = (int)max(e, 1u) - 150 + shift;
    const uint32_t r = (uint32_t)min(max(39 - s, 0), 63);
    const uint32_t t = (uint32_t)min(max(s, 0), 63);
    const uint64_t lo = ((uint64_t)m << 39) >> r;
    const uint64_t hi = (uint64_t)m << t;
    return s > 39 ? hi : lo;
}

// fixed_weight when s <= 39 is known: a <= alpha_max with alpha_max a normal
// float and shift = 63 - L - E chosen from alpha_max (2^(E-1) <= alpha_max <
// 2^E) give s <= 39 - L.
__device__ __forceinline__ uint64_t fixed_weight_le39(float a, int shift)
{
    const uint32_t b = __float_as_uint(a);
    const uint32_t e = (b >> 23) & 0xFFu;
    const uint32_t m = (b & 0x7FFFFFu) | (min(e, 1u) << 23);
    const int s = (int)max(e, 1u) - 150 + shift;
    return ((uint64_t)m << 39) >> (uint32_t)min(39 - s, 63);
}

// (float)S rounded to nearest even, then scaled by 2^-shift with one more
// rounding -- the value ldexpf((float)S, -shift) takes.
__device__ __forceinline__ float fixed_to_float(uint64_t S, int shift)
{
    if (S == 0) return 0.0f;
    const int n = 64 - __clzll((long long)S);
    uint64_t q = S;
    int r = 0;
    if (n > 24) {
        r = n - 24;
        q = S >> r;
        const uint64_t rem = S & ((1ull << r) - 1);
        const uint64_t half = 1ull << (r - 1);
        if (rem > half || (rem == half && (q & 1))) q += 1;
        if (q == (1ull << 24)) {
            q >>= 1;
            r += 1;
        }
    }
    return ldexpf((float)(uint32_t)q, r - shift);
}

__device__ __forceinline__ uint64_t umul64hi(uint64_t a, uint64_t b)
{
    return __umul64hi(a, b);
}

}  // namespace arsel
