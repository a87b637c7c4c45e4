// Context management and error strings of the C ABI.
#include <math.h>
#include <new>
#include <string.h>

#include "launch.hpp"

extern "C" int arsel_create(arsel_ctx **out, int device)
{
    if (!out) return ARSEL_ERR_NULL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return ARSEL_ERR_HIP;
    if (device < 0 || device >= n) return ARSEL_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return ARSEL_ERR_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return ARSEL_ERR_DEVICE;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return ARSEL_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return ARSEL_ERR_DEVICE;

    arsel_ctx *c = new (std::nothrow) arsel_ctx();
    if (!c) return ARSEL_ERR_ALLOC;
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    // Two dense tiles per compute unit (160 KB of LDS on gfx950).
    c->tile_lds_bytes = std::min<size_t>(c->lds_per_block, 80 * 1024);
    c->dense_tile = 16;
    c->dense_waves = 0;        // automatic (see launch_tile)
    c->trial_lanes = 0;
    c->sched.wave_max_m = 1024;   // the tuner's usual choice on log-uniform sizes
    c->sched.block_waves = 8;
    c->sched.lds_max_m = 0;       // hard piece 16380 floats
    c->sched.blocks_per_cu = 4;
    c->queue = nullptr;
    c->order = nullptr;
    c->order_bytes = 0;
    c->order_dev = nullptr;
    c->order_dev_bytes = 0;
    c->staging = nullptr;
    c->staging_bytes = 0;
    c->staging_event = nullptr;
    c->mlp_fused = 0;
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->ssa_tab = nullptr;
    c->ssa_tab_bytes = 0;
    c->ln_tab = nullptr;
    c->scratch = nullptr;
    double tab[2 * (kLnTabHi - kLnTabLo + 1)];
    for (int i = kLnTabLo; i <= kLnTabHi; ++i) {
        tab[2 * (i - kLnTabLo)] = log((double)i / 128.0);
        tab[2 * (i - kLnTabLo) + 1] = 128.0 / (double)i;
    }
    c->order_split = -1;
    c->order_items = c->order_large = c->order_waves = 0;
    c->inst = nullptr;
    c->inst_bytes = 0;
    if (hipMalloc((void **)&c->queue, kQueueBytes) != hipSuccess ||
        hipMemset(c->queue, 0, kQueueBytes) != hipSuccess ||
        hipMalloc((void **)&c->ln_tab, sizeof(tab)) != hipSuccess ||
        hipMemcpy(c->ln_tab, tab, sizeof(tab), hipMemcpyHostToDevice) != hipSuccess) {
        if (c->queue) (void)hipFree(c->queue);
        if (c->ln_tab) (void)hipFree(c->ln_tab);
        delete c;
        (void)hipSetDevice(prev);
        return ARSEL_ERR_ALLOC;
    }
    // the no-allocation ragged call finds its scratch here, once per context,
    // with the context's device current; a failure only disables that call
    if (arsel::ragged_scratch_address(&c->scratch) != ARSEL_OK) c->scratch = nullptr;
    (void)hipSetDevice(prev);
    *out = c;
    return ARSEL_OK;
}

extern "C" int arsel_destroy(arsel_ctx *ctx)
{
    if (!ctx) return ARSEL_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    if (ctx->queue) (void)hipFree(ctx->queue);
    if (ctx->order) (void)hipFree(ctx->order);
    if (ctx->order_dev) (void)hipFree(ctx->order_dev);
    if (ctx->inst) (void)hipFree(ctx->inst);
    for (void *p : ctx->retired) (void)hipFree(p);
    if (ctx->staging_event) {
        (void)hipEventSynchronize(ctx->staging_event);
        (void)hipEventDestroy(ctx->staging_event);
    }
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->ssa_tab) (void)hipFree(ctx->ssa_tab);
    if (ctx->ln_tab) (void)hipFree(ctx->ln_tab);
    (void)hipSetDevice(prev);
    delete ctx;
    return ARSEL_OK;
}

extern "C" const char *arsel_strerror(int code)
{
    switch (code) {
    case ARSEL_OK: return "ok";
    case ARSEL_ERR_NULL: return "a required pointer is NULL";
    case ARSEL_ERR_SIZE: return "invalid size (M < 1, K < 0 or beyond the 32-bit range)";
    case ARSEL_ERR_LAYOUT: return "layout must be ARSEL_AOS or ARSEL_SOA";
    case ARSEL_ERR_LD: return "leading dimension too small for the layout";
    case ARSEL_ERR_HIP: return "a HIP call or kernel launch failed";
    case ARSEL_ERR_DEVICE: return "bad device id, or the device is not gfx950";
    case ARSEL_ERR_ALLOC: return "allocation failed";
    case ARSEL_ERR_ARG: return "invalid argument";
    default: return "unknown error";
    }
}

extern "C" int arsel_get_schedule(arsel_ctx *ctx, arsel_schedule *out)
{
    if (!ctx || !out) return ARSEL_ERR_NULL;
    *out = ctx->sched;
    return ARSEL_OK;
}

extern "C" int arsel_set_schedule(arsel_ctx *ctx, const arsel_schedule *s)
{
    if (!ctx || !s) return ARSEL_ERR_NULL;
    const int bw = s->block_waves;
    if (!(bw == 4 || bw == 8 || bw == 16)) return ARSEL_ERR_ARG;
    if (s->wave_max_m < 1 || s->lds_max_m < 0 || s->blocks_per_cu < 1 || s->blocks_per_cu > 8)
        return ARSEL_ERR_ARG;
    // the pick launch's wavefront slices; the hard piece (at most 16380
    // floats) is checked with the launch
    const size_t lds = (size_t)bw * s->wave_max_m * sizeof(float);
    if (lds + 2048 > ctx->lds_per_block) return ARSEL_ERR_ARG;
    ctx->sched = *s;
    return ARSEL_OK;
}

extern "C" int arsel_set_dense_config(arsel_ctx *ctx, int32_t tile, int32_t waves)
{
    if (!ctx) return ARSEL_ERR_NULL;
    if (tile == 0 && waves == 0) {          // back to the automatic choice
        ctx->dense_tile = 16;
        ctx->dense_waves = 0;
        return ARSEL_OK;
    }
    if (tile < 1 || tile > 64) return ARSEL_ERR_ARG;
    if (!(waves == 4 || waves == 8 || waves == 16)) return ARSEL_ERR_ARG;
    ctx->dense_tile = tile;
    ctx->dense_waves = waves;
    return ARSEL_OK;
}
