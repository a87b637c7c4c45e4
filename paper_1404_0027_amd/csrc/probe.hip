// Read-bandwidth probe: what the device delivers on an array read once with
// the selection kernels' own 16-byte non-temporal loads, all issued before
// any is consumed.  A kernel's bandwidth is then reported against this
// achievable ceiling as well as the data-sheet peak.  Not part of the
// selection method.
#include "launch.hpp"
#include "device.hpp"

namespace arsel {

constexpr int kProbeWaves = 16;
constexpr int kProbeThreads = kProbeWaves * 64;
constexpr int kProbeBatch = 4;   // float4 loads per thread per workgroup (contiguous mode)
constexpr int kProbeTileBatch = 6;

// Contiguous span of n4 float4: workgroup b reads slots [b * NT * kProbeBatch, ...).
__global__ __launch_bounds__(kProbeThreads) void k_probe_span(const float *p, int64_t n4,
                                                              uint32_t *sink)
{
    __shared__ uint32_t red[kProbeWaves];
    const int64_t base = (int64_t)blockIdx.x * kProbeThreads * kProbeBatch + threadIdx.x;
    f32x4 v[kProbeBatch];
#pragma unroll
    for (int u = 0; u < kProbeBatch; ++u) {
        const int64_t i = base + (int64_t)u * kProbeThreads;
        v[u] = i < n4 ? load_stream4(p + 4 * i) : (f32x4){0.f, 0.f, 0.f, 0.f};
    }
    uint32_t m = 0;
#pragma unroll
    for (int u = 0; u < kProbeBatch; ++u) {
        m = max(m, __float_as_uint(v[u].x));
        m = max(m, __float_as_uint(v[u].y));
        m = max(m, __float_as_uint(v[u].z));
        m = max(m, __float_as_uint(v[u].w));
    }
    m = wave_max_u32(m);
    if (lane_id() == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t r = 0;
        for (int w = 0; w < kProbeWaves; ++w) r = max(r, red[w]);
        sink[blockIdx.x] = r;
    }
}

// The dense SoA tile pattern: workgroup b (remapped per XCD) reads columns
// [tile * b', tile * b' + tile) of every one of `rows` rows (row stride ld),
// a lane taking 4 consecutive columns of one row, kProbeTileBatch loads in
// flight per thread.
__global__ __launch_bounds__(kProbeThreads) void k_probe_tile(const float *p, int32_t rows,
                                                              int64_t ld, int32_t tile,
                                                              uint32_t *sink)
{
    __shared__ uint32_t red[kProbeWaves];
    const int tid = threadIdx.x;
    const int k0 = xcd_tile(blockIdx.x, gridDim.x) * tile;
    const int qpr = tile >> 2;
    const int qshift = __builtin_ctz(qpr);
    const int total = rows * qpr;
    const int row_step = kProbeThreads >> qshift;
    const int j0 = tid >> qshift, q = tid & (qpr - 1);
    const float *src = p + k0 + 4 * q;
    uint32_t m = 0;
    for (int base = 0; base < total; base += kProbeTileBatch * kProbeThreads) {
        f32x4 v[kProbeTileBatch];
#pragma unroll
        for (int u = 0; u < kProbeTileBatch; ++u)
            if (base + u * kProbeThreads + tid < total)
                v[u] = load_stream4(src + (int64_t)(j0 + ((base >> qshift) + u * row_step)) * ld);
#pragma unroll
        for (int u = 0; u < kProbeTileBatch; ++u)
            if (base + u * kProbeThreads + tid < total) {
                m = max(m, __float_as_uint(v[u].x));
                m = max(m, __float_as_uint(v[u].y));
                m = max(m, __float_as_uint(v[u].z));
                m = max(m, __float_as_uint(v[u].w));
            }
    }
    m = wave_max_u32(m);
    if (lane_id() == 0) red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        uint32_t r = 0;
        for (int w = 0; w < kProbeWaves; ++w) r = max(r, red[w]);
        sink[blockIdx.x] = r;
    }
}

}  // namespace arsel

using namespace arsel;

extern "C" int arsel_probe_read(arsel_ctx *ctx, const float *p, int32_t rows, int32_t cols,
                                int64_t ld, int32_t tile, uint32_t *sink, int64_t sink_len,
                                int64_t *grid_out, void *stream)
{
    if (!ctx || !grid_out) return ARSEL_ERR_NULL;
    *grid_out = 0;
    if (rows < 0 || cols < 0) return ARSEL_ERR_SIZE;
    if (ld < cols || (ld % 4) != 0) return ARSEL_ERR_LD;
    if (tile != 0 && (tile < 4 || tile > 64 || (tile & (tile - 1)) != 0 || cols % tile != 0))
        return ARSEL_ERR_ARG;
    if (tile == 0 && cols != ld) return ARSEL_ERR_LD;
    const int64_t n4 = (int64_t)rows * ld / 4;
    const int64_t per = (int64_t)kProbeThreads * kProbeBatch;
    const int64_t grid = tile == 0 ? (n4 + per - 1) / per : cols / tile;
    *grid_out = grid;
    if (grid == 0) return ARSEL_OK;
    if (grid > 0x7FFFFFFF) return ARSEL_ERR_SIZE;
    if (!p || !sink) return ARSEL_ERR_NULL;
    if (((uintptr_t)p % 16) != 0) return ARSEL_ERR_ARG;
    if (sink_len < grid) return ARSEL_ERR_SIZE;
    int rc = ctx_activate(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (tile == 0)
        hipLaunchKernelGGL(k_probe_span, dim3((unsigned)grid), dim3(kProbeThreads), 0, s, p, n4, sink);
    else
        hipLaunchKernelGGL(k_probe_tile, dim3((unsigned)grid), dim3(kProbeThreads), 0, s, p, rows, ld,
                           tile, sink);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}
