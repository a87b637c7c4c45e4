// Host-side context shared by the entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/arsel.h"

// Bytes of the context's queue word array.
constexpr size_t kQueueBytes = 2048;

struct arsel_ctx {
    int device;
    int num_cu;
    size_t lds_per_block;     // device limit on LDS per workgroup (bytes)
    size_t tile_lds_bytes;    // LDS budget of one dense tile
    int dense_tile;           // instances per dense tile (upper bound)
    int dense_waves;          // wavefronts per dense workgroup (4, 8, 16; 0: automatic)
    int trial_lanes;          // lanes per instance of the broadcast kernel (0: automatic)
    arsel_schedule sched;     // ragged schedule
    uint32_t *queue;          // kQueueBytes of device counters of the uneven-batch call (list
                              // lengths, per-class histograms of the device-built lists)
    int32_t *order;           // host-built work lists of the ragged kernel (reused while the
    size_t order_bytes;       // sizes repeat), grown on demand
    int32_t *order_dev;       // device-built work lists (rebuilt by every call that uses
    size_t order_dev_bytes;   // them, graph replays included), grown on demand
    std::vector<void *> retired;   // buffers replaced by larger ones: kept until
                                   // arsel_destroy, so graphs captured earlier stay valid
    std::vector<int64_t> order_sizes;   // host sizes the work lists were built from,
    int32_t order_split;                // for this wave_max_m (-1: lists not reusable)
    uint32_t order_items, order_large, order_waves;   // their lengths (scan items, large
                                                       // instances, small instances)
    void *inst;               // per-instance scan accumulators of the uneven-batch call (bit
    size_t inst_bytes;        // maximum, float sum), zero between calls, grown on demand
    int32_t *staging;         // pinned host staging of the work lists
    size_t staging_bytes;
    hipEvent_t staging_event; // completion of the last staging copy
    int mlp_fused;            // inference forward by the fused kernel when the shape allows
    void *ws;                 // MLP workspace (activations, gradients), grown on demand
    size_t ws_bytes;
    void *ssa_tab;            // packed dependency rows of the SSA run, grown on demand
    size_t ssa_tab_bytes;
    double *ln_tab;           // {ln(i/128), 128/i} for i = 96..192 (the run's logarithm)
    void *scratch;            // this device's address of the static scratch array of
                              // arsel_select_ragged_noalloc (null if it could not be found)
};

// Grid of the run's table-driven logarithm: c_i = i / 128, i in [96, 192].
constexpr int kLnTabLo = 96, kLnTabHi = 192;

namespace arsel {

// Broadcast selection with packed rounds (select_packed.hip): K instances of
// one vector, uniform proposal (Q null) or integer proposal Q.
int launch_packed(arsel_ctx *ctx, const float *alpha, const uint32_t *Q, int32_t M, int32_t K,
                  uint64_t seed, uint64_t step, uint32_t t_max, int32_t *index, float *alpha0,
                  uint32_t *trials, hipStream_t s);

// LDS bytes the broadcast kernel needs for M reactions: alpha; with a
// proposal also Q, its prefix and a guide table of 2^ceil(log2 M) entries.
inline size_t packed_lds_bytes(int32_t M, bool proposal)
{
    if (!proposal) return (size_t)M * sizeof(float);
    size_t t = 1;
    while (t < (size_t)M) t <<= 1;
    return ((size_t)M * 3 + t) * sizeof(uint32_t);
}

// Address of the static scratch array of arsel_select_ragged_noalloc on the
// current device (select_ragged.hip).
int ragged_scratch_address(void **out);

// Grow a context-owned device buffer to at least `need` bytes (contents not
// kept).  The old buffer is retired, not freed: a graph captured earlier may
// still hold its address, so it is released only by arsel_destroy.  Growth is
// geometric, which bounds the retired memory by the final size.
inline int ctx_grow(arsel_ctx *ctx, void **p, size_t *cap, size_t need)
{
    if (*cap >= need) return ARSEL_OK;
    const size_t want = std::max(need, 2 * *cap);
    void *q = nullptr;
    if (hipMalloc(&q, want) != hipSuccess) {
        (void)hipGetLastError();
        return ARSEL_ERR_ALLOC;
    }
    if (*p) {
        try {
            ctx->retired.push_back(*p);
        } catch (...) {
            (void)hipFree(q);
            return ARSEL_ERR_ALLOC;
        }
    }
    *p = q;
    *cap = want;
    return ARSEL_OK;
}

inline int ctx_activate(arsel_ctx *ctx)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return ARSEL_ERR_HIP;
    if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return ARSEL_ERR_DEVICE;
    return ARSEL_OK;
}

}  // namespace arsel
