// Host-side context shared by the entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/arsel.h"

struct arsel_ctx {
    int device;
    int num_cu;
    size_t lds_per_block;     // device limit on LDS per workgroup (bytes)
    size_t tile_lds_bytes;    // LDS budget of one dense tile
    int dense_tile;           // instances per dense tile (upper bound)
    int dense_waves;          // wavefronts per dense workgroup (4, 8, 16)
    arsel_schedule sched;     // ragged schedule
    uint32_t *queue;          // device counters of the persistent ragged kernel (4 x u32)
    int32_t *order;           // device work lists of the ragged kernel, grown on demand
    size_t order_bytes;
    int32_t *staging;         // pinned host staging of the work lists
    size_t staging_bytes;
    hipEvent_t staging_event; // completion of the last staging copy
    void *ws;                 // MLP workspace (activations, gradients), grown on demand
    size_t ws_bytes;
};

namespace arsel {

inline int ctx_activate(arsel_ctx *ctx)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return ARSEL_ERR_HIP;
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return ARSEL_ERR_DEVICE;
    return ARSEL_OK;
}

}  // namespace arsel
