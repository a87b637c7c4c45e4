// Wavefront reductions on DPP row shifts and row broadcasts (no LDS traffic,
// unlike the ds_bpermute behind __shfl_xor): the pattern of
// wave_incl_scan_u32, so lane 63 ends with the total and is read back.
#pragma once

#include "device.hpp"

namespace arsel {

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x)
{
    const uint32_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)x);
    const uint32_t hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(x >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t readlane63_u64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Sum of 32-bit integers (wrapping, so signed values sum exactly while the
// total fits); every lane returns it.
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan_u32(x), 63);
}

// Binary64 sum in the tree order of the row scan (lanes with no source add
// +0.0); every lane returns it.
__device__ __forceinline__ double wave_sum_f64_dpp(double x)
{
    auto bits = [](double v) { return (uint64_t)__double_as_longlong(v); };
    auto dbl = [](uint64_t b) { return __longlong_as_double((long long)b); };
    x += dbl(dpp_u64<0x111>(bits(x)));          // row_shr:1
    x += dbl(dpp_u64<0x112>(bits(x)));          // row_shr:2
    x += dbl(dpp_u64<0x114>(bits(x)));          // row_shr:4
    x += dbl(dpp_u64<0x118>(bits(x)));          // row_shr:8
    x += dbl(dpp_u64<0x142, 0xA>(bits(x)));     // row_bcast:15 into rows 1 and 3
    x += dbl(dpp_u64<0x143, 0xC>(bits(x)));     // row_bcast:31 into rows 2 and 3
    return dbl(readlane63_u64(bits(x)));
}

// Binary64 sum of lanes 0..15 (row 0) by row shifts; every lane returns it.
__device__ __forceinline__ double row0_sum_f64(double x)
{
    auto bits = [](double v) { return (uint64_t)__double_as_longlong(v); };
    auto dbl = [](uint64_t b) { return __longlong_as_double((long long)b); };
    x += dbl(dpp_u64<0x111>(bits(x)));          // row_shr:1
    x += dbl(dpp_u64<0x112>(bits(x)));          // row_shr:2
    x += dbl(dpp_u64<0x114>(bits(x)));          // row_shr:4
    x += dbl(dpp_u64<0x118>(bits(x)));          // row_shr:8 -> lane 15: sum of the row
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bits(x), 15);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(bits(x) >> 32), 15);
    return dbl((uint64_t)lo | ((uint64_t)hi << 32));
}

// Maximum of non-negative binary64 values (+0.0 is the identity); every
// lane returns it.
__device__ __forceinline__ double wave_max_f64_nonneg(double x)
{
    auto bits = [](double v) { return (uint64_t)__double_as_longlong(v); };
    auto dbl = [](uint64_t b) { return __longlong_as_double((long long)b); };
    x = fmax(x, dbl(dpp_u64<0x111>(bits(x))));
    x = fmax(x, dbl(dpp_u64<0x112>(bits(x))));
    x = fmax(x, dbl(dpp_u64<0x114>(bits(x))));
    x = fmax(x, dbl(dpp_u64<0x118>(bits(x))));
    x = fmax(x, dbl(dpp_u64<0x142, 0xA>(bits(x))));
    x = fmax(x, dbl(dpp_u64<0x143, 0xC>(bits(x))));
    return dbl(readlane63_u64(bits(x)));
}

// Maximum of non-negative floats: their bit order is their value order.
__device__ __forceinline__ float wave_max_f32_nonneg(float x)
{
    return __uint_as_float(wave_max_u32(__float_as_uint(x)));
}

// Fetch-and-add of a wave-uniform v by the wavefront: the first active lane
// alone performs the atomic and every active lane gets its old value.  (An
// atomic issued by every lane with a per-lane value -- v on one lane, 0 on
// the others -- is compiled into a scan over the active lanes, one lane per
// iteration, several hundred instructions per call.)  Does not depend on
// which lanes are active.
__device__ __forceinline__ uint32_t wave_claim_add(uint32_t *p, uint32_t v)
{
    const uint32_t leader = (uint32_t)__builtin_amdgcn_readfirstlane((int)lane_id());
    uint32_t old = 0;
    if ((uint32_t)lane_id() == leader) old = atomicAdd(p, v);
    return (uint32_t)__builtin_amdgcn_readlane((int)old, (int)leader);
}

}  // namespace arsel
