// Uneven batches in one persistent launch.
//
// Instance k has M_k = offsets[k+1] - offsets[k] reactions (AoS).  The
// instances are split into two work lists: large ones (M > wave_max_m) are
// run by a whole workgroup (staged in LDS when M <= lds_max_m, otherwise
// gathered from global memory right after the streaming pass that computes
// the maximum), small ones by a single wavefront.  Persistent workgroups
// take items from the two lists through atomic counters, the large list
// first; both lists are ordered longest first by power-of-two size class (on
// the host when the caller passes the sizes, else by a one-workgroup counting
// sort on the device).  The schedule (wave_max_m, waves per workgroup, lds_max_m, workgroups per CU) is
// chosen by the autotuner and never changes the results: every instance
// gets the same trial stream and rule as arsel_select with instance id k.
#include <algorithm>

#include "launch.hpp"
#include "select_block.hpp"
#include "wave_reduce.hpp"

namespace arsel {

struct RaggedArgs {
    const float *alpha;
    const int64_t *offsets;
    const int32_t *list_block;   // instance ids of the workgroup list
    const int32_t *list_wave;    // instance ids of the wavefront list
    const uint32_t *counts;      // device list lengths (device-built lists), or null
    uint32_t n_block, n_wave;    // host list lengths (host-built lists)
    uint32_t *queue;             // [0] workgroup list cursor, [1] wavefront list cursor,
                                 // [2], [3] device list lengths, [4] finished workgroups
    int32_t *index;
    float *alpha0;
    uint32_t *trials;
    uint64_t seed, step;
    uint32_t t_max;
    int32_t lds_max_m;
    int32_t wave_max_m;
};

// Size class of an instance: floor(log2 M) (0 for M <= 1, negative sizes included).
__device__ __forceinline__ int size_class(int64_t m)
{
    return m <= 1 ? 0 : 63 - __clzll((long long)m);
}

// Device-side split of the instances into the two lists, ordered longest first
// by size class (a counting sort in one workgroup), for batches of at most
// kOrderMaxK instances.  The kernel also sets the counters of the launch that
// follows: both cursors and the finished-workgroup count to zero, the list
// lengths to the counts.  It reads nothing the previous call left, so a call
// that stopped with an error after enqueuing it leaves no state behind.
constexpr int32_t kOrderMaxK = 1 << 16;
constexpr int kOrderThreads = 1024;

__global__ __launch_bounds__(kOrderThreads) void k_ragged_order(const int64_t *offsets, int32_t K,
                                                                int32_t wave_max_m,
                                                                int32_t *list_block,
                                                                int32_t *list_wave, uint32_t *queue)
{
    __shared__ uint32_t cnt[2][64];
    __shared__ uint32_t pos[2][64];
    const int tid = threadIdx.x;
    if (tid < 128) cnt[tid >> 6][tid & 63] = 0;
    __syncthreads();
    for (int k = tid; k < K; k += kOrderThreads) {
        const int64_t m = offsets[k + 1] - offsets[k];
        atomicAdd(&cnt[m > wave_max_m][size_class(m)], 1u);
    }
    __syncthreads();
    if (tid < 2) {
        uint32_t run = 0;
        for (int b = 63; b >= 0; --b) {
            pos[tid][b] = run;
            run += cnt[tid][b];
        }
        queue[2 + (tid == 0)] = run;      // queue[2]: workgroup list, queue[3]: wavefront list
        if (tid == 0) {
            queue[0] = 0;
            queue[1] = 0;
            queue[4] = 0;
        }
    }
    __syncthreads();
    for (int k = tid; k < K; k += kOrderThreads) {
        const int64_t m = offsets[k + 1] - offsets[k];
        const int l = m > wave_max_m;
        const uint32_t p = atomicAdd(&pos[l][size_class(m)], 1u);
        (l ? list_block : list_wave)[p] = k;
    }
}

// Counters of the launch that follows set to zero (larger device-built batches).
__global__ void k_ragged_reset(uint32_t *queue)
{
    if (threadIdx.x < 5) queue[threadIdx.x] = 0;
}

// Device-side split of the instances into the two lists (order arbitrary);
// the counters start at zero (k_ragged_reset runs first).
__global__ void k_ragged_classify(const int64_t *offsets, int32_t K, int32_t wave_max_m,
                                  int32_t *list_block, int32_t *list_wave, uint32_t *counts)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int64_t m = offsets[k + 1] - offsets[k];
    if (m > wave_max_m)
        list_block[atomicAdd(&counts[0], 1u)] = k;
    else
        list_wave[atomicAdd(&counts[1], 1u)] = k;
}

// Device-built work lists and counters for a launch of k_select_ragged.
static int build_lists_on_device(const int64_t *offsets, int32_t K, int32_t wave_max_m,
                                 int32_t *list_block, int32_t *list_wave, uint32_t *queue,
                                 hipStream_t s)
{
    if (K <= kOrderMaxK) {
        hipLaunchKernelGGL(k_ragged_order, dim3(1), dim3(kOrderThreads), 0, s, offsets, K,
                           wave_max_m, list_block, list_wave, queue);
    } else {
        hipLaunchKernelGGL(k_ragged_reset, dim3(1), dim3(64), 0, s, queue);
        if (hipGetLastError() != hipSuccess) return ARSEL_ERR_HIP;
        hipLaunchKernelGGL(k_ragged_classify, dim3((K + 255) / 256), dim3(256), 0, s, offsets, K,
                           wave_max_m, list_block, list_wave, queue + 2);
    }
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

__device__ __forceinline__ void ragged_write(const RaggedArgs &a, int k, const Outcome &o)
{
    a.index[k] = o.index;
    if (a.alpha0) a.alpha0[k] = o.alpha0;
    if (a.trials) a.trials[k] = o.trials;
}

// Sizes that cannot be processed (negative, or beyond 32-bit indexing).
__device__ __forceinline__ bool bad_size(int64_t m)
{
    return m < 0 || m > 0x7FFFFFFF;
}

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_select_ragged(RaggedArgs a)
{
    extern __shared__ float lds[];
    __shared__ BlockScratch<NW> bs;
    __shared__ uint32_t item;
    constexpr int NT = NW * 64;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = lane_id();
    const uint32_t n_block = uniform_u32(a.counts ? a.counts[0] : a.n_block);
    const uint32_t n_wave = uniform_u32(a.counts ? a.counts[1] : a.n_wave);
    const bool want_a0 = a.alpha0 != nullptr;

    // Large instances: the whole workgroup per instance.  The next item is
    // claimed as soon as the current one starts (the atomic's latency then
    // overlaps the current item) and published through LDS at its end.
    if (tid == 0) item = atomicAdd(&a.queue[0], 1u);
    for (;;) {
        __syncthreads();
        const uint32_t i = uniform_u32(item);
        __syncthreads();
        if (i >= n_block) break;
        const uint32_t claimed = tid == 0 ? atomicAdd(&a.queue[0], 1u) : 0u;
        const int k = a.list_block[i];
        const int64_t off = a.offsets[k];
        const int64_t m64 = a.offsets[k + 1] - off;
        if (bad_size(m64) || m64 == 0) {
            if (tid == 0) {
                Outcome o;
                o.index = m64 == 0 ? -1 : -2;
                o.alpha0 = m64 == 0 ? 0.0f : __builtin_nanf("");
                o.trials = 0;
                ragged_write(a, k, o);
                item = claimed;
            }
            continue;
        }
        const uint32_t M = (uint32_t)m64;
        const float *row = a.alpha + off;
        const bool staged = (int64_t)M <= (int64_t)a.lds_max_m;
        // one streaming pass: bit-maximum (validity + alpha_max), staging into LDS
        uint32_t mb = stream_bitmax<NT>(row, M, staged ? lds : nullptr, tid);
        mb = block_max_u32<NW>(mb, bs);   // its barriers also publish the staged row
        const Stream st = make_stream(a.seed, a.step, (uint32_t)k, kTagUniform);
        const uint32_t hint = mb < 0x7F800000u ? mb : 0xFFFFFFFFu;
        Outcome o;
        if (staged)
            o = block_select<NW>(ContigAcc{lds}, M, hint, st, a.t_max, want_a0, bs);
        else
            o = block_select<NW>(ContigAcc{row}, M, hint, st, a.t_max, want_a0, bs, row, lds,
                                 (uint32_t)max(a.lds_max_m, NW * a.wave_max_m));
        if (tid == 0) {
            ragged_write(a, k, o);
            item = claimed;
        }
    }

    // Small instances: one wavefront per instance, staged in the wave's LDS slice.
    float *slice = lds + (size_t)wave * a.wave_max_m;
    // Same prefetch of the next item, per wavefront: the claim's old value
    // stays in a register until the current item is done.
    uint32_t claim = wave_claim_add(&a.queue[1], 1u);
    for (;;) {
        const uint32_t i = uniform_u32(claim);
        if (i >= n_wave) break;
        claim = wave_claim_add(&a.queue[1], 1u);
        const int k = a.list_wave[i];
        const int64_t off = a.offsets[k];
        const int64_t m64 = a.offsets[k + 1] - off;
        Outcome o;
        if (bad_size(m64) || m64 == 0 || m64 > a.wave_max_m) {
            o.index = m64 == 0 ? -1 : -2;
            o.alpha0 = m64 == 0 ? 0.0f : __builtin_nanf("");
            o.trials = 0;
        } else {
            const uint32_t M = (uint32_t)m64;
            const float *row = a.alpha + off;
            const uint32_t mb = wave_max_u32(stream_bitmax<kWave>(row, M, slice, lane));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const Stream st = make_stream(a.seed, a.step, (uint32_t)k, kTagUniform);
            o = wave_select_hint(ContigAcc{slice}, M, mb, st, a.t_max, want_a0);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (lane == 0) ragged_write(a, k, o);
    }

    // The last workgroup to finish clears the counters for the next call
    // (every other workgroup's list claims are done by then).
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(&a.queue[4], 1u) == gridDim.x - 1) {
            __threadfence();
            for (int c = 0; c < 5; ++c) a.queue[c] = 0;
        }
    }
}

template <int NW>
static int launch_ragged(arsel_ctx *ctx, const RaggedArgs &a, size_t lds, hipStream_t s)
{
    const int grid = ctx->num_cu * ctx->sched.blocks_per_cu;
    hipLaunchKernelGGL(k_select_ragged<NW>, dim3(grid), dim3(NW * 64), lds, s, a);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

// Scratch of arsel_select_ragged_noalloc: the launch counters (padded to
// 256 bytes) and the two work lists of at most kNoAllocMaxK instances, in a
// file-scope device array.  Each GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (ragged_scratch_address).
constexpr int32_t kNoAllocMaxK = kOrderMaxK;
constexpr size_t kScratchQueueWords = 64;
static __device__ __align__(256) uint32_t scratch[kScratchQueueWords + 2 * (size_t)kNoAllocMaxK];

int ragged_scratch_address(void **out)
{
    *out = nullptr;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return ARSEL_ERR_HIP;
    }
    *out = p;
    return ARSEL_OK;
}


}  // namespace arsel

using namespace arsel;

extern "C" int arsel_select_ragged(arsel_ctx *ctx, const float *alpha, const int64_t *offsets,
                                   int32_t K, const int64_t *host_sizes, uint64_t seed,
                                   uint64_t step, uint32_t t_max, int32_t *index, float *alpha0,
                                   uint32_t *trials, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    if (K < 0) return ARSEL_ERR_SIZE;
    if (K == 0) return ARSEL_OK;
    if (!alpha || !offsets || !index) return ARSEL_ERR_NULL;
    int rc = ctx_activate(ctx);
    if (rc) return rc;
    (void)hipGetLastError();   // a stale error of earlier work is not this call's
    const arsel_schedule &sc = ctx->sched;
    const int nw = sc.block_waves;
    const size_t lds = std::max<size_t>((size_t)sc.lds_max_m, (size_t)nw * sc.wave_max_m) * sizeof(float);
    if (lds > ctx->lds_per_block - 2048) return ARSEL_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    // Under graph capture the lists are built on the device, inside the graph,
    // in their own buffer: a replay then depends on no list a later call
    // leaves in the context.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return ARSEL_ERR_HIP;
    if (cap != hipStreamCaptureStatusNone) host_sizes = nullptr;
    const size_t list_bytes = 2 * (size_t)K * sizeof(int32_t);
    int32_t *lists;
    if (host_sizes) {
        const int32_t *held = ctx->order;
        rc = ctx_grow(ctx, (void **)&ctx->order, &ctx->order_bytes, list_bytes);
        if (rc || ctx->order != held) ctx->order_split = -1;
        if (rc) return rc;
        lists = ctx->order;
    } else {
        if ((rc = ctx_grow(ctx, (void **)&ctx->order_dev, &ctx->order_dev_bytes, list_bytes)))
            return rc;
        lists = ctx->order_dev;
    }

    RaggedArgs a;
    a.alpha = alpha;
    a.offsets = offsets;
    a.list_block = lists;
    a.list_wave = lists + K;
    a.queue = ctx->queue;
    a.index = index;
    a.alpha0 = alpha0;
    a.trials = trials;
    a.seed = seed;
    a.step = step;
    a.t_max = t_max;
    a.lds_max_m = sc.lds_max_m;
    a.wave_max_m = sc.wave_max_m;

    // Host-built lists: the counters are zero, cleared at creation and by the
    // last workgroup of every launch of the kernel (a call that returns an
    // error launches no kernel that touches them).  Device-built lists: the
    // ordering kernel sets the counters itself.
    if (host_sizes) {
        // The lists depend only on the sizes and the split: a call with the
        // sizes and split of the lists already on the device reuses them.
        const bool same = ctx->order_split == sc.wave_max_m && ctx->order_sizes.size() == (size_t)K &&
                          std::equal(host_sizes, host_sizes + K, ctx->order_sizes.begin());
        if (!same) {
            ctx->order_split = -1;
            // Longest first within each list; the lists go to the device through a
            // pinned staging buffer (reused once the previous copy has finished).
            // Counting sort on floor(log2 M) (O(K)): sizes within a factor 2 keep
            // their order, larger buckets first.
            const size_t bytes = 2 * (size_t)K * sizeof(int32_t);
            if (ctx->staging_event && hipEventSynchronize(ctx->staging_event) != hipSuccess)
                return ARSEL_ERR_HIP;
            if (ctx->staging_bytes < bytes) {
                if (ctx->staging && hipHostFree(ctx->staging) != hipSuccess) return ARSEL_ERR_HIP;
                ctx->staging = nullptr;
                ctx->staging_bytes = 0;
                if (hipHostMalloc((void **)&ctx->staging, bytes, hipHostMallocDefault) != hipSuccess)
                    return ARSEL_ERR_ALLOC;
                ctx->staging_bytes = bytes;
            }
            auto bucket = [&](int32_t k) {
                const int64_t m = host_sizes[k];
                return m <= 1 ? 0 : 63 - __builtin_clzll((unsigned long long)m);
            };
            auto large = [&](int32_t k) { return host_sizes[k] > sc.wave_max_m; };
            size_t nb[2][64] = {};
            for (int32_t k = 0; k < K; ++k) ++nb[large(k)][bucket(k)];
            size_t start[2][64];
            size_t len[2] = {0, 0};
            for (int l = 0; l < 2; ++l)
                for (int b = 63; b >= 0; --b) {
                    start[l][b] = len[l];
                    len[l] += nb[l][b];
                }
            int32_t *list[2] = {ctx->staging + K, ctx->staging};   // wavefront, workgroup
            for (int32_t k = 0; k < K; ++k) {
                const int l = large(k);
                list[l][start[l][bucket(k)]++] = k;
            }
            if (hipMemcpyAsync(ctx->order, ctx->staging, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
                return ARSEL_ERR_HIP;
            if (!ctx->staging_event && hipEventCreateWithFlags(&ctx->staging_event, hipEventDisableTiming) != hipSuccess)
                return ARSEL_ERR_HIP;
            if (hipEventRecord(ctx->staging_event, s) != hipSuccess) return ARSEL_ERR_HIP;
            ctx->order_blocks = (uint32_t)len[1];
            ctx->order_waves = (uint32_t)len[0];
            try {
                ctx->order_sizes.assign(host_sizes, host_sizes + K);
                ctx->order_split = sc.wave_max_m;
            } catch (...) {
                ctx->order_sizes.clear();   // the lists stay valid for this call only
            }
        }
        a.counts = nullptr;
        a.n_block = ctx->order_blocks;
        a.n_wave = ctx->order_waves;
    } else {
        if ((rc = build_lists_on_device(offsets, K, sc.wave_max_m, lists, lists + K, ctx->queue, s)))
            return rc;
        a.counts = ctx->queue + 2;
        a.n_block = a.n_wave = 0;
    }
    switch (nw) {
    case 4: return launch_ragged<4>(ctx, a, lds, s);
    case 8: return launch_ragged<8>(ctx, a, lds, s);
    case 16: return launch_ragged<16>(ctx, a, lds, s);
    default: return ARSEL_ERR_ARG;
    }
}

// The same selection with the work lists built on the device in the GPU's
// static scratch array: no allocation of any kind.  k_ragged_order sets every
// counter before the selection kernel reads it, so nothing left in the array
// by an earlier call (or an interrupted one) is read.
extern "C" int arsel_select_ragged_noalloc(arsel_ctx *ctx, const float *alpha,
                                           const int64_t *offsets, int32_t K, uint64_t seed,
                                           uint64_t step, uint32_t t_max, int32_t *index,
                                           float *alpha0, uint32_t *trials, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    if (K < 0 || K > kNoAllocMaxK) return ARSEL_ERR_SIZE;
    if (K == 0) return ARSEL_OK;
    if (!alpha || !offsets || !index) return ARSEL_ERR_NULL;
    if (!ctx->scratch) return ARSEL_ERR_HIP;
    int rc = ctx_activate(ctx);
    if (rc) return rc;
    (void)hipGetLastError();   // a stale error of earlier work is not this call's
    const arsel_schedule &sc = ctx->sched;
    const int nw = sc.block_waves;
    const size_t lds = std::max<size_t>((size_t)sc.lds_max_m, (size_t)nw * sc.wave_max_m) * sizeof(float);
    if (lds > ctx->lds_per_block - 2048) return ARSEL_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;

    uint32_t *queue = static_cast<uint32_t *>(ctx->scratch);
    int32_t *lists = reinterpret_cast<int32_t *>(queue + kScratchQueueWords);
    RaggedArgs a;
    a.alpha = alpha;
    a.offsets = offsets;
    a.list_block = lists;
    a.list_wave = lists + K;
    a.counts = queue + 2;
    a.n_block = a.n_wave = 0;
    a.queue = queue;
    a.index = index;
    a.alpha0 = alpha0;
    a.trials = trials;
    a.seed = seed;
    a.step = step;
    a.t_max = t_max;
    a.lds_max_m = sc.lds_max_m;
    a.wave_max_m = sc.wave_max_m;
    hipLaunchKernelGGL(k_ragged_order, dim3(1), dim3(kOrderThreads), 0, s, offsets, K,
                       sc.wave_max_m, lists, lists + K, queue);
    if (hipGetLastError() != hipSuccess) return ARSEL_ERR_HIP;
    switch (nw) {
    case 4: return launch_ragged<4>(ctx, a, lds, s);
    case 8: return launch_ragged<8>(ctx, a, lds, s);
    case 16: return launch_ragged<16>(ctx, a, lds, s);
    default: return ARSEL_ERR_ARG;
    }
}
