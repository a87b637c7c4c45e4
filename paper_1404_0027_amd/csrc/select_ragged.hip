// Uneven batches: instance k has M_k = offsets[k+1] - offsets[k] reactions
// at alpha[offsets[k] ..] (AoS).  Four launches per call:
//
//  1. k_ragged_scan streams the instances with M_k > wave_max_m (nearly all
//     the bytes) as work items of at most a few thousand elements dealt to
//     the wavefronts round-robin, two load batches in flight per wavefront
//     and no barrier: the same access pattern as a plain streaming read.
//     Each item adds its bit-maximum (which certifies validity and is
//     alpha_max) and a float sum of its elements to the instance's slot.
//  2. k_ragged_split estimates each such instance's expected number of trials
//     M alpha_max / alpha_0 from the slot (the estimate only schedules;
//     results never depend on it), lists the instances expected to need more
//     than kHardTrials trials as hard, cut into chunks of one LDS piece, and
//     the others as easy.
//  3. k_ragged_hard takes the hard chunks, dealt to the workgroups
//     round-robin: each stages its chunk in LDS, draws the instance's trials
//     and tests those whose candidate lies in the chunk, and records the
//     least accepted trial (an atomic minimum per instance) and the chunk's
//     exact fixed-point sum.  A hard row is thus read once more, at streaming
//     speed, and no candidate costs a DRAM sector.
//  4. k_ragged_pick, one wavefront per instance: hard instances take the
//     least accepted trial, or the exact fallback located from the chunk
//     sums; easy instances run their trials gathering candidates from global
//     memory (the rows were just streamed); small instances (M_k <=
//     wave_max_m) stream their row into the wave's LDS slice and select there.
//
// Every instance gets the same trial stream and rule as arsel_select with
// instance id k, so results do not depend on the schedule, the chunking or
// the estimate.
#include <algorithm>

#include "launch.hpp"
#include "select_block.hpp"
#include "wave_reduce.hpp"

namespace arsel {

// One chunk of a large instance (16 bytes); positions relative to offsets[0].
struct RScan {
    int64_t start;
    int32_t len;
    int32_t k;
};

// Per-instance accumulator of the scan: bit-maximum and float sum.
struct RAcc {
    uint32_t maxbits;
    float sum;
};

constexpr int kScanBatch = 8;                       // float4 per lane per load batch
constexpr int64_t kScanChunk = 64 * kScanBatch * 4; // elements per chunk (nominal): one batch
constexpr int kScanWaves = 4;                       // wavefronts per scan workgroup
constexpr int kScanBlocksPerCU = 4;            // 16 wavefronts per CU at ~108 VGPRs
constexpr uint32_t kHardTrials = 512;               // expected trials above which a workgroup selects
constexpr int kListAlignInts = 8;                   // 32-byte alignment between list sections

// Chunk plan of an instance at element offset off with m elements: chunks of
// L elements counted from the multiple of 4 at or below off, L the larger of
// kScanChunk and m / maxch (rounded up to 4), so at most maxch + 1 chunks.
struct ChunkPlan {
    int64_t a0, L;
    int32_t nch;
};

__host__ __device__ inline ChunkPlan chunk_plan(int64_t off, int64_t m, int32_t maxch)
{
    ChunkPlan p;
    p.a0 = off & ~(int64_t)3;
    int64_t L = (m + maxch - 1) / maxch;
    L = (L + 3) & ~(int64_t)3;
    p.L = L > kScanChunk ? L : kScanChunk;
    p.nch = (int32_t)((off + m - p.a0 + p.L - 1) / p.L);
    return p;
}

__host__ __device__ inline RScan chunk_item(const ChunkPlan &p, int64_t off, int64_t m, int32_t k, int32_t c)
{
    RScan it;
    const int64_t s = p.a0 + p.L * c;
    const int64_t e = s + p.L;
    it.start = s > off ? s : off;
    it.len = (int32_t)((e < off + m ? e : off + m) - it.start);
    it.k = k;
    return it;
}

// Size class of an instance: floor(log2 M) (0 for M <= 1, negative sizes included).
__host__ __device__ inline int size_class(int64_t m)
{
    return m <= 1 ? 0 : 63 - __builtin_clzll((unsigned long long)m);
}

// Sizes that cannot be processed (negative, or beyond 32-bit indexing).
__host__ __device__ inline bool bad_size(int64_t m)
{
    return m < 0 || m > 0x7FFFFFFF;
}

// Counters in the context's queue word array.  The list lengths the split
// kernel counts are zeroed by the scan kernel of the same call; the device
// ordering kernels set their own.
enum : int {
    kQNHard = 0,      // hard list length (split kernel)
    kQNEasy = 1,      // easy list length (split kernel)
    kQNHItems = 2,    // hard chunks (split kernel)
    kQNSmall = 3,     // small list length (device-built lists)
    kQNItems = 4,     // scan items (device-built lists)
    kQNLarge = 5,     // large list length (device-built lists)
    kQWords = 6
};

// Device-built lists, ordered longest first by size class like the host
// ones, for any K, in three launches: k_list_clear zeroes the per-class
// histograms and cursors in the queue words, k_list_count adds each block's
// histograms to them, and k_list_scatter places each instance at its class's
// start (from the histograms) plus its block's share of the class (one global
// atomic per block and non-empty class) plus its rank in the block.  The
// order within a class depends on the atomics; nothing downstream depends on
// that order.  k_list_scatter also sets the list lengths.
constexpr int kListThreads = 256;
constexpr int kClasses = 64;
enum : int {
    kQHist = 64,                          // [3][64] counts: small, large, scan items
    kQCursor = kQHist + 3 * kClasses,     // [3][64] next free slot per class
    kQueueWordsAll = kQCursor + 3 * kClasses
};

__global__ void k_list_clear(uint32_t *queue)
{
    for (int i = threadIdx.x; i < kQueueWordsAll; i += blockDim.x) queue[i] = 0;
}

__global__ __launch_bounds__(kListThreads) void k_list_count(const int64_t *offsets, int32_t K,
                                                             int32_t wave_max_m, int32_t maxch,
                                                             uint32_t *queue)
{
    __shared__ uint32_t h[3 * kClasses];
    const int t = threadIdx.x;
    for (int i = t; i < 3 * kClasses; i += kListThreads) h[i] = 0;
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * kListThreads + t;
    if (k < K) {
        const int64_t base = offsets[0];
        const int64_t o0 = offsets[k];
        const int64_t m = offsets[k + 1] - o0;
        const int c = size_class(m);
        if (m <= wave_max_m || bad_size(m)) {
            atomicAdd(&h[c], 1u);
        } else {
            atomicAdd(&h[kClasses + c], 1u);
            atomicAdd(&h[2 * kClasses + c], (uint32_t)chunk_plan(o0 - base, m, maxch).nch);
        }
    }
    __syncthreads();
    for (int i = t; i < 3 * kClasses; i += kListThreads)
        if (h[i]) atomicAdd(&queue[kQHist + i], h[i]);
}

__global__ __launch_bounds__(kListThreads) void k_list_scatter(const int64_t *offsets, int32_t K,
                                                               int32_t wave_max_m, int32_t maxch,
                                                               int32_t *small, int32_t *large,
                                                               RScan *items, uint32_t *queue)
{
    __shared__ uint32_t start[3 * kClasses];   // first position of each class in its list
    __shared__ uint32_t loc[3 * kClasses];     // this block's count, then its base, per class
    const int t = threadIdx.x;
    for (int i = t; i < 3 * kClasses; i += kListThreads) {
        start[i] = queue[kQHist + i];
        loc[i] = 0;
    }
    __syncthreads();
    if (t < 3) {
        uint32_t run = 0;
        for (int b = kClasses - 1; b >= 0; --b) {
            const uint32_t n = start[t * kClasses + b];
            start[t * kClasses + b] = run;
            run += n;
        }
        if (blockIdx.x == 0) queue[t == 0 ? kQNSmall : t == 1 ? kQNLarge : kQNItems] = run;
    }
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * kListThreads + t;
    const bool in = k < K;
    int c = 0;
    bool sm = false;
    uint32_t r = 0, ri = 0;
    int64_t off = 0, m = 0;
    ChunkPlan p{0, 0, 0};
    if (in) {
        const int64_t o0 = offsets[k];
        m = offsets[k + 1] - o0;
        off = o0 - offsets[0];
        c = size_class(m);
        sm = m <= wave_max_m || bad_size(m);
        if (sm) {
            r = atomicAdd(&loc[c], 1u);
        } else {
            p = chunk_plan(off, m, maxch);
            r = atomicAdd(&loc[kClasses + c], 1u);
            ri = atomicAdd(&loc[2 * kClasses + c], (uint32_t)p.nch);
        }
    }
    __syncthreads();
    for (int i = t; i < 3 * kClasses; i += kListThreads)
        if (loc[i]) loc[i] = atomicAdd(&queue[kQCursor + i], loc[i]);
    __syncthreads();
    if (in) {
        if (sm) {
            small[start[c] + loc[c] + r] = (int32_t)k;
        } else {
            large[start[kClasses + c] + loc[kClasses + c] + r] = (int32_t)k;
            const uint32_t q = start[2 * kClasses + c] + loc[2 * kClasses + c] + ri;
            for (int32_t ch = 0; ch < p.nch; ++ch) items[q + ch] = chunk_item(p, off, m, (int32_t)k, ch);
        }
    }
}

// The counters only (the error path of a call).
__global__ void k_ragged_reset(uint32_t *queue)
{
    if (threadIdx.x < kQWords) queue[threadIdx.x] = 0;
}

__global__ void k_ragged_clear(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// A scan item's elements: the unaligned head, a 16-byte aligned body of
// float4 slots loaded kScanBatch per lane at a time, and the tail.
struct ChunkSpan {
    int64_t hs, be;   // aligned body [hs, be)
    int32_t nq;       // float4 slots in the body
    int32_t nb;       // load batches (at least 1)
};

__device__ __forceinline__ ChunkSpan chunk_span(const float *base, const RScan &it)
{
    const int64_t s = it.start, e = it.start + it.len;
    const int64_t head = (int64_t)((4 - (((uintptr_t)(base + s) >> 2) & 3)) & 3);
    ChunkSpan c;
    c.hs = min(s + head, e);
    c.nq = (int32_t)((e - c.hs) >> 2);
    c.be = c.hs + 4 * (int64_t)c.nq;
    constexpr int per = 64 * kScanBatch;
    c.nb = c.nq > per ? (c.nq + per - 1) / per : 1;
    return c;
}

// One load batch of a wavefront: body slots [b per, (b + 1) per), the head in
// batch 0 and the tail in the last batch, all issued before any is used.
struct WaveLoads {
    f32x4 v[kScanBatch];
    float hx, tx;

    __device__ __forceinline__ void issue(const float *base, const RScan &it, const ChunkSpan &c,
                                          int b, int lane)
    {
        const int64_t s = it.start, e = it.start + it.len;
        const float *b4 = base + c.hs;
        const int q0 = b * 64 * kScanBatch;
#pragma unroll
        for (int u = 0; u < kScanBatch; ++u) {
            const int q = q0 + u * 64 + lane;
            if (q < c.nq) v[u] = load_stream4(b4 + 4 * (int64_t)q);
        }
        hx = (b == 0 && lane < c.hs - s) ? base[s + lane] : 0.0f;
        tx = (b == c.nb - 1 && lane < e - c.be) ? base[c.be + lane] : 0.0f;
    }

    __device__ __forceinline__ void consume(const RScan &it, const ChunkSpan &c, int b, int lane,
                                            uint32_t &mb, float &sum) const
    {
        const int64_t s = it.start, e = it.start + it.len;
        const int q0 = b * 64 * kScanBatch;
#pragma unroll
        for (int u = 0; u < kScanBatch; ++u) {
            if (q0 + u * 64 + lane < c.nq) {
                mb = max(mb, __float_as_uint(v[u].x));
                mb = max(mb, __float_as_uint(v[u].y));
                mb = max(mb, __float_as_uint(v[u].z));
                mb = max(mb, __float_as_uint(v[u].w));
                sum += (v[u].x + v[u].y) + (v[u].z + v[u].w);
            }
        }
        if (b == 0 && lane < c.hs - s) {
            mb = max(mb, __float_as_uint(hx));
            sum += hx;
        }
        if (b == c.nb - 1 && lane < e - c.be) {
            mb = max(mb, __float_as_uint(tx));
            sum += tx;
        }
    }
};

__device__ __forceinline__ float wave_sum_f32(float x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// Wavefront w of the grid takes items w, w + W, w + 2 W, ... (W wavefronts in
// the grid); the next batch (of this item or the next) is always in flight
// while the current one is reduced.
__global__ __launch_bounds__(kScanWaves * 64) void k_ragged_scan(const float *alpha,
                                                                 const int64_t *offsets,
                                                                 const RScan *items,
                                                                 const uint32_t *n_items_dev,
                                                                 uint32_t n_items_host, RAcc *acc,
                                                                 uint32_t *queue)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) queue[kQNHard] = queue[kQNEasy] = queue[kQNHItems] = 0;
    const int lane = lane_id();
    const uint32_t W = gridDim.x * kScanWaves;
    uint32_t g = blockIdx.x * kScanWaves + (threadIdx.x >> 6);
    const uint32_t n = uniform_u32(n_items_dev ? *n_items_dev : n_items_host);
    const float *base = alpha + offsets[0];
    if (g >= n) return;
    RScan it = items[g];
    ChunkSpan cs = chunk_span(base, it);
    int b = 0;
    WaveLoads ld[2];
    ld[0].issue(base, it, cs, 0, lane);
    uint32_t mb = 0;
    float sum = 0.0f;
    // the batch after (it, b): its item, span and batch index
    auto next = [&](RScan &ni, ChunkSpan &ns, int &nbi, uint32_t &ng) -> bool {
        if (nbi + 1 < ns.nb) {
            ++nbi;
            return true;
        }
        ng += W;
        if (ng >= n) return false;
        ni = items[ng];
        ns = chunk_span(base, ni);
        nbi = 0;
        return true;
    };
    for (;;) {
        // slot 0 holds (it, b); issue the following batch into slot 1
        RScan it1 = it;
        ChunkSpan cs1 = cs;
        int b1 = b;
        uint32_t g1 = g;
        const bool more = next(it1, cs1, b1, g1);
        if (more) ld[1].issue(base, it1, cs1, b1, lane);
        ld[0].consume(it, cs, b, lane, mb, sum);
        if (!more || g1 != g) {
            const uint32_t m = wave_max_u32(mb);
            const float ssum = wave_sum_f32(sum);
            if (lane == 0) {
                atomicMax(&acc[it.k].maxbits, m);
                atomicAdd(&acc[it.k].sum, ssum);
            }
            mb = 0;
            sum = 0.0f;
        }
        if (!more) break;
        it = it1;
        cs = cs1;
        b = b1;
        g = g1;
        // the same with the slots swapped
        it1 = it;
        cs1 = cs;
        b1 = b;
        g1 = g;
        const bool more2 = next(it1, cs1, b1, g1);
        if (more2) ld[0].issue(base, it1, cs1, b1, lane);
        ld[1].consume(it, cs, b, lane, mb, sum);
        if (!more2 || g1 != g) {
            const uint32_t m = wave_max_u32(mb);
            const float ssum = wave_sum_f32(sum);
            if (lane == 0) {
                atomicMax(&acc[it.k].maxbits, m);
                atomicAdd(&acc[it.k].sum, ssum);
            }
            mb = 0;
            sum = 0.0f;
        }
        if (!more2) break;
        it = it1;
        cs = cs1;
        b = b1;
        g = g1;
    }
}

constexpr int kHardWaves = 8;                        // wavefronts of a chunk workgroup

// One chunk of a hard instance: chunk c of instance k (elements [c L, (c+1) L)
// of its row, L = hard_chunk_len), and the fixed-point sums of its weights
// taken by each wavefront of the chunk kernel.  For a chunk of one piece
// these are the sums over the wavefronts' ranges of PieceLoads, in order;
// for a longer chunk only their total means anything.
struct HItem {
    int32_t k;
    int32_t c;
    uint64_t wsum[kHardWaves];
};
constexpr int kHardThreads = kHardWaves * kWave;
constexpr uint32_t kHardPieceMax = kHardThreads * kStreamBatch * 4 - 4;   // one load batch, any alignment
constexpr uint32_t kHardPieceMin = (uint32_t)kScanChunk;
constexpr int kHardPer = 4;                          // Philox blocks per thread and round
constexpr uint32_t kHardRound = 2u * kHardThreads * kHardPer;   // trials per round

// Floats of a hard row staged in LDS at a time, from the schedule's lds_max_m
// (0 selects the largest).
__host__ __device__ inline uint32_t hard_piece(int32_t lds_max_m)
{
    if (lds_max_m <= 0) return kHardPieceMax;
    const uint32_t p = (uint32_t)lds_max_m & ~3u;
    return p < kHardPieceMin ? kHardPieceMin : (p > kHardPieceMax ? kHardPieceMax : p);
}

// Chunk length of a hard instance of m elements: the piece, or m / maxch
// (rounded up to 4) when longer, so at most maxch chunks; never shorter than
// the instance's scan items, so the hard chunks never outnumber them.
__host__ __device__ inline uint32_t hard_chunk_len(int64_t m, int32_t maxch, uint32_t piece)
{
    int64_t L = (m + maxch - 1) / maxch;
    L = (L + 3) & ~(int64_t)3;
    return (uint32_t)(L > (int64_t)piece ? L : (int64_t)piece);
}

// Hard / easy split of the large instances by the expected number of trials
// M alpha_max / alpha_0 (estimated).  Hard instance at position p of its list
// owns chunks hc[p] .. hc[p] + ceil(M / L) - 1, and its slot in `best` is
// reset.  Rows whose scan found an invalid value, no positive sum or a
// subnormal maximum go to the easy list, whose wavefront path validates the
// row itself.  Positions come
// from one atomic per wavefront and counter (the counters start at zero), so
// the lists are in no particular order.
constexpr int kSplitThreads = 256;

__global__ __launch_bounds__(kSplitThreads) void k_ragged_split(const int64_t *offsets, const int32_t *large,
                                                                const uint32_t *n_large_dev,
                                                                uint32_t n_large_host, const RAcc *acc,
                                                                int32_t maxch, uint32_t piece,
                                                                int32_t *hard, int32_t *easy,
                                                                HItem *hitems, uint32_t *hc,
                                                                unsigned long long *best,
                                                                uint32_t *queue)
{
    const uint32_t n = n_large_dev ? *n_large_dev : n_large_host;
    const uint32_t i = blockIdx.x * kSplitThreads + threadIdx.x;
    const int lane = lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const bool in = i < n;
    bool is_hard = false;
    int k = 0;
    uint32_t nch = 0;
    if (in) {
        k = large[i];
        const RAcc a = acc[k];
        const int64_t m = offsets[k + 1] - offsets[k];
        const float amax = __uint_as_float(a.maxbits);
        // a hard row needs a normal maximum (its chunks take the cheaper exact
        // weight); a subnormal one, like an invalid row, goes to the easy list
        const bool valid = a.maxbits >= 0x00800000u && a.maxbits < 0x7F800000u && a.sum > 0.0f;
        is_hard = valid && (float)m * amax > (float)kHardTrials * a.sum;
        if (is_hard) {
            const uint32_t L = hard_chunk_len(m, maxch, piece);
            nch = (uint32_t)((m + L - 1) / L);
        }
    }
    const uint64_t mh = __ballot(is_hard), me = __ballot(in && !is_hard);
    const uint32_t cincl = wave_incl_scan_u32(nch);
    const uint32_t ctot = readlane_u32(cincl, kWave - 1);
    uint32_t bh = 0, be = 0, bc = 0;
    if (lane == 0) {
        if (mh) bh = atomicAdd(&queue[kQNHard], (uint32_t)__popcll(mh));
        if (me) be = atomicAdd(&queue[kQNEasy], (uint32_t)__popcll(me));
        if (ctot) bc = atomicAdd(&queue[kQNHItems], ctot);
    }
    bh = readlane_u32(bh, 0);
    be = readlane_u32(be, 0);
    bc = readlane_u32(bc, 0);
    if (is_hard) {
        const uint32_t p = bh + (uint32_t)__popcll(mh & below);
        const uint32_t c0 = bc + cincl - nch;
        hard[p] = k;
        hc[p] = c0;
        best[k] = kNoAccept;
        for (uint32_t c = 0; c < nch; ++c) {
            hitems[c0 + c].k = k;
            hitems[c0 + c].c = (int32_t)c;
        }
    } else if (in) {
        easy[be + (uint32_t)__popcll(me & below)] = k;
    }
}

// Where a hard chunk lies: instance k, its row, and the chunk [c0, ce).
struct ChunkRef {
    int k;
    uint32_t M, c0, ce;
    const float *row;
};

__device__ __forceinline__ ChunkRef chunk_ref(const HItem *hitems, const int64_t *offsets, const float *alpha,
                                              uint32_t it, int32_t maxch, uint32_t piece)
{
    ChunkRef r;
    r.k = (int)uniform_u32((uint32_t)hitems[it].k);
    const uint32_t c = uniform_u32((uint32_t)hitems[it].c);
    const int64_t off = offsets[r.k];
    const int64_t m = offsets[r.k + 1] - off;
    r.M = (uint32_t)m;
    r.row = alpha + off;
    const uint32_t L = hard_chunk_len(m, maxch, piece);
    r.c0 = c * L;
    r.ce = min(r.M, r.c0 + L);
    return r;
}

// The hard chunks, dealt to the workgroups round-robin.  A chunk's elements
// pass through LDS `piece` floats at a time (one piece unless the chunk is
// longer); for each piece the thread draws its share of the instance's trials
// (Philox blocks tid + NT q of the round, the first round while the piece's
// loads are in flight) and tests those whose candidate lies in the piece.
// Rounds of kHardRound trials continue only while no trial of the chunk
// below the next round has been accepted.  The chunk's least accepted trial
// goes to the instance's slot by an atomic minimum, and each wavefront's
// fixed-point sum to the item.  A trial's outcome does not depend on which chunk tests it,
// so the least over all chunks is the sequential rule's first acceptance.
// The loads of the next piece (of this chunk or the next) are issued as soon
// as the current piece is in LDS, so they are in flight while it is tested.
__global__ __launch_bounds__(kHardThreads, 4) void k_ragged_hard(const float *alpha, const int64_t *offsets,
                                                              HItem *hitems, const uint32_t *queue,
                                                              const RAcc *acc, unsigned long long *best,
                                                              int32_t maxch, uint32_t piece,
                                                              uint64_t seed, uint64_t step,
                                                              uint32_t t_max)
{
    extern __shared__ float buf[];
    __shared__ BlockScratch<kHardWaves> bs;
    constexpr int NT = kHardThreads;
    const uint32_t tid = threadIdx.x;
    const uint32_t n_items = uniform_u32(queue[kQNHItems]);
    const uint32_t nblocks = (uint32_t)(((uint64_t)t_max + 1) / 2);   // Philox blocks of t_max trials
    uint32_t it = blockIdx.x;
    if (it >= n_items) return;
    ChunkRef cur = chunk_ref(hitems, offsets, alpha, it, maxch, piece);
    uint32_t p0 = cur.c0;
    PieceLoads<NT> ld;
    ld.issue(cur.row, cur.ce, p0, piece, tid);
    if (tid == 0) bs.key = kNoAccept;
    uint64_t part = 0;
    uint64_t kb = kNoAccept;   // least accepted (trial << 32 | j) of this thread in the chunk
    uint32_t held = 0xFFFFFFFFu;   // round whose draws the registers hold
    uint32_t ja[kHardPer], jb[kHardPer], ua[kHardPer], ub[kHardPer];
    for (;;) {
        const uint32_t n = min(piece, cur.ce - p0);
        const bool last_piece = p0 + piece >= cur.ce;
        // the unit after this one, its position read early
        uint32_t nit = it, np0 = p0 + piece;
        ChunkRef nxt = cur;
        bool have_next = true;
        if (last_piece) {
            nit = it + gridDim.x;
            have_next = nit < n_items;
            if (have_next) {
                nxt = chunk_ref(hitems, offsets, alpha, nit, maxch, piece);
                np0 = nxt.c0;
            }
        }
        const float amax = __uint_as_float(uniform_u32(acc[cur.k].maxbits));
        const int shift = 63 - ceil_log2_u32(cur.M) - exponent_above(amax);
        const double envs = (double)amax * 0x1p-32;
        const uint32_t thresh = lemire_threshold(cur.M);
        const Stream st = make_stream(seed, step, (uint32_t)cur.k, kTagUniform);
        auto draw = [&](uint32_t round) {
            held = round;
#pragma unroll
            for (int q = 0; q < kHardPer; ++q) {
                uint32_t b = round * (NT * kHardPer) + tid + NT * q;
                // the counter is chunk-invariant: keep the compiler from hoisting
                // its Philox products out of the chunk loop (they spilled)
                asm volatile("" : "+v"(b));
                ja[q] = jb[q] = 0xFFFFFFFFu;
                ua[q] = ub[q] = 0;
                if (b < nblocks) {
                    const Words w = st.block(b);
                    uint32_t j;
                    if (lemire(w.w0, cur.M, thresh, j) && 2 * b < t_max) ja[q] = j;
                    if (lemire(w.w2, cur.M, thresh, j) && 2 * b + 1 < t_max) jb[q] = j;
                    ua[q] = w.w1;
                    ub[q] = w.w3;
                }
                // one block's temporaries live at a time
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        // a later piece of the same chunk reuses the first round's draws
        if (p0 == cur.c0 || held != 0) draw(0);
        // hard rows have a normal maximum (the split's rule), so every weight
        // has s <= 39
        part += ld.template store<true>(cur.row, cur.ce, p0, piece, tid, buf, shift);
        __syncthreads();
        if (have_next) ld.issue(nxt.row, nxt.ce, np0, piece, tid);
        for (uint32_t round = 0;;) {
#pragma unroll
            for (int q = 0; q < kHardPer; ++q) {
                const uint32_t b = round * (NT * kHardPer) + tid + NT * q;
                if (ja[q] - p0 < n && (double)ua[q] * envs < (double)buf[ja[q] - p0])
                    kb = min(kb, ((uint64_t)(2 * b) << 32) | ja[q]);
                if (jb[q] - p0 < n && (double)ub[q] * envs < (double)buf[jb[q] - p0])
                    kb = min(kb, ((uint64_t)(2 * b + 1) << 32) | jb[q]);
                __builtin_amdgcn_sched_barrier(0);
            }
            ++round;
            if ((uint64_t)round * kHardRound >= t_max) break;
            if (kb != kNoAccept) atomicMin((unsigned long long *)&bs.key, (unsigned long long)kb);
            __syncthreads();
            const uint64_t sofar = uniform_u64(bs.key);
            if (sofar < ((uint64_t)round * kHardRound << 32)) break;
            draw(round);
        }
        if (last_piece && kb != kNoAccept) atomicMin((unsigned long long *)&bs.key, (unsigned long long)kb);
        __syncthreads();   // the piece buffer is refilled next; bs.key is complete
        if (last_piece) {
            part = wave_sum_u64(part);
            if ((tid & (kWave - 1)) == 0) hitems[it].wsum[tid >> 6] = part;
            if (tid == 0) {
                const uint64_t key = bs.key;
                if (key != kNoAccept) atomicMin(&best[cur.k], (unsigned long long)key);
                bs.key = kNoAccept;
            }
            part = 0;
            kb = kNoAccept;
        }
        if (!have_next) break;
        cur = nxt;
        p0 = np0;
        it = nit;
    }
}

// Least j in [0, n) whose inclusive prefix of F_j = floor(p[j] 2^shift)
// exceeds target (which must be below the n weights' sum; -1 otherwise), by
// one wavefront reading 16-byte slots eight per lane at a time.
__device__ int32_t wave_search_span(const float *p, uint32_t n, int shift, uint64_t target)
{
    const int lane = lane_id();
    const uint32_t align = (uint32_t)(((16 - ((uintptr_t)p & 15)) & 15) >> 2);
    const uint32_t head = align < n ? align : n;
    uint64_t f = (uint32_t)lane < head ? fixed_weight(p[lane], shift) : 0;
    uint64_t incl = wave_incl_scan_u64(f);
    uint64_t hit = __ballot((uint32_t)lane < head && incl > target);
    if (hit) return first_lane(hit);
    uint64_t carry = readlane_u64(incl, kWave - 1);
    const uint32_t nq = (n - head) >> 2;
    const float *s4 = p + head;
    constexpr int B = 8;
    for (uint32_t b0 = 0; b0 < nq; b0 += kWave * B) {
        f32x4 v[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t i = b0 + u * kWave + lane;
            v[u] = i < nq ? *reinterpret_cast<const f32x4 *>(s4 + 4 * i) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const uint32_t i = b0 + u * kWave + lane;
            const uint64_t f0 = fixed_weight(v[u].x, shift), f1 = fixed_weight(v[u].y, shift);
            const uint64_t f2 = fixed_weight(v[u].z, shift), f3 = fixed_weight(v[u].w, shift);
            const uint64_t sum4 = (f0 + f1) + (f2 + f3);
            incl = carry + wave_incl_scan_u64(sum4);
            hit = __ballot(i < nq && incl > target);
            if (hit) {
                const int src = first_lane(hit);
                const uint64_t e = incl - sum4;   // this lane's exclusive prefix
                const uint32_t r = e + f0 > target ? 0u : e + f0 + f1 > target ? 1u : e + f0 + f1 + f2 > target ? 2u : 3u;
                return (int32_t)(head + 4 * (b0 + u * kWave + (uint32_t)src) + readlane_u32(r, src));
            }
            carry = readlane_u64(incl, kWave - 1);
        }
    }
    const uint32_t t0 = head + 4 * nq;
    f = (uint32_t)lane < n - t0 ? fixed_weight(p[t0 + lane], shift) : 0;
    incl = carry + wave_incl_scan_u64(f);
    hit = __ballot((uint32_t)lane < n - t0 && incl > target);
    return hit ? (int32_t)(t0 + first_lane(hit)) : -1;
}

struct PickArgs {
    const float *alpha;
    const int64_t *offsets;
    const int32_t *hard, *easy, *small;
    const HItem *hitems;             // hard chunks with their sums
    const uint32_t *hc;              // [n_hard] first chunk of each hard instance
    const unsigned long long *best;  // [K] least accepted key of each hard instance
    RAcc *acc;                       // [K] scan results; each large instance's is cleared when picked
    const uint32_t *n_small_dev;     // device small-list length, or null
    uint32_t n_small_host;
    uint32_t *queue;
    int32_t *index;
    float *alpha0;
    uint32_t *trials;
    uint64_t seed, step;
    uint32_t t_max;
    int32_t maxch;                   // chunk plan of the hard instances
    uint32_t piece;
    int32_t wave_max_m;
};

__device__ __forceinline__ void pick_write(const PickArgs &a, int k, const Outcome &o)
{
    a.index[k] = o.index;
    if (a.alpha0) a.alpha0[k] = o.alpha0;
    if (a.trials) a.trials[k] = o.trials;
}

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_ragged_pick(PickArgs a)
{
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = lane_id();
    const bool want_a0 = a.alpha0 != nullptr;
    const uint32_t n_hard = uniform_u32(a.queue[kQNHard]);
    const uint32_t n_easy = uniform_u32(a.queue[kQNEasy]);
    const uint32_t n_small = uniform_u32(a.n_small_dev ? *a.n_small_dev : a.n_small_host);
    const uint32_t gw = blockIdx.x * NW + (uint32_t)wave, nwaves = gridDim.x * NW;

    // Work is dealt round-robin, with no shared counter: a same-address
    // atomic per claim serialises at the memory side (measured ~15 ns each,
    // about as long as the whole selection for ~10^4 claims).
    // Hard instances: the chunk kernel's least accepted trial, else the
    // fallback's target located from the chunk sums and searched in its chunk.
    for (uint32_t i = gw; i < n_hard; i += nwaves) {
        const int k = a.hard[i];
        const int64_t off = a.offsets[k];
        const int64_t m = a.offsets[k + 1] - off;
        const uint32_t M = (uint32_t)m;
        const uint64_t key = uniform_u64(a.best[k]);
        const uint32_t L = hard_chunk_len(m, a.maxch, a.piece);
        const uint32_t h0 = uniform_u32(a.hc[i]);
        const uint32_t h1 = h0 + (uint32_t)((m + L - 1) / L);
        const float amax = __uint_as_float(uniform_u32(a.acc[k].maxbits));
        const int shift = 63 - ceil_log2_u32(M) - exponent_above(amax);
        Outcome o;
        o.alpha0 = 0.0f;
        uint64_t S = 0;
        if (key == kNoAccept || want_a0) {
            for (uint32_t x = lane; x < (h1 - h0) * kHardWaves; x += kWave)
                S += a.hitems[h0 + x / kHardWaves].wsum[x % kHardWaves];
            S = wave_sum_u64(S);
            if (want_a0) o.alpha0 = fixed_to_float(S, shift);
        }
        if (key != kNoAccept) {
            o.index = (int32_t)(uint32_t)key;
            o.trials = (uint32_t)(key >> 32) + 1;
        } else {
            const Stream st = make_stream(a.seed, a.step, (uint32_t)k, kTagUniform);
            const Words w = st.block(kFallbackBlock);
            const uint64_t V = (uint64_t)w.w0 | ((uint64_t)w.w1 << 32);
            const uint64_t target = umul64hi(V, S);
            // the chunk holding the target, from the chunk totals
            uint32_t hit_c = h1 - 1;
            uint64_t before = 0, carry = 0;
            for (uint32_t h = h0; h < h1; h += kWave) {
                const uint32_t x = h + (uint32_t)lane;
                uint64_t s = 0;
                if (x < h1)
#pragma unroll
                    for (int v = 0; v < kHardWaves; ++v) s += a.hitems[x].wsum[v];
                const uint64_t incl = carry + wave_incl_scan_u64(s);
                const uint64_t hit = __ballot(x < h1 && incl > target);
                if (hit) {
                    const int src = first_lane(hit);
                    hit_c = h + (uint32_t)src;
                    before = readlane_u64(incl - s, src);
                    break;
                }
                carry = readlane_u64(incl, kWave - 1);
            }
            const uint32_t c0 = (hit_c - h0) * L;
            const uint32_t cn = min(L, M - c0);
            const float *crow = a.alpha + off + c0;
            uint32_t lo = 0, hi = cn;
            if (L <= a.piece) {
                // one piece: the wavefront range holding the target
                using PL = PieceLoads<kHardThreads>;
                const PL::Span sp = PL::span(a.alpha + off, M, c0, a.piece);
                const uint64_t ws = lane < kHardWaves ? a.hitems[hit_c].wsum[lane] : 0;
                const uint64_t incl = wave_incl_scan_u64(ws);
                const uint64_t hit = __ballot(lane < kHardWaves && incl > target - before);
                const int wv = hit ? first_lane(hit) : kHardWaves - 1;
                before += readlane_u64(incl - ws, wv);
                lo = PL::wave_begin(sp, (uint32_t)wv);
                hi = wv + 1 < kHardWaves ? PL::wave_begin(sp, (uint32_t)wv + 1) : sp.n;
            }
            const int32_t j = wave_search_span(crow + lo, hi - lo, shift, target - before);
            o.index = (int32_t)(c0 + lo) + j;
            o.trials = a.t_max + 1;
        }
        if (lane == 0) {
            pick_write(a, k, o);
            a.acc[k] = RAcc{0u, 0.0f};
        }
    }

    // Easy instances: one wavefront each, gathering from global memory, dealt
    // from the last wavefront down (the first ones took the hard instances).
    for (uint32_t i = nwaves - 1 - gw; i < n_easy; i += nwaves) {
        const int k = a.easy[i];
        const int64_t off = a.offsets[k];
        const uint32_t M = (uint32_t)(a.offsets[k + 1] - off);
        const uint32_t mb = uniform_u32(a.acc[k].maxbits);
        const Stream st = make_stream(a.seed, a.step, (uint32_t)k, kTagUniform);
        const Outcome o = wave_select_hint(ContigAcc{a.alpha + off}, M, mb, st, a.t_max, want_a0);
        if (lane == 0) {
            pick_write(a, k, o);
            a.acc[k] = RAcc{0u, 0.0f};
        }
    }
    // Small instances: one wavefront each, staged in the wave's LDS slice.
    float *slice = lds + (size_t)wave * a.wave_max_m;
    for (uint32_t i = gw; i < n_small; i += nwaves) {
        const int k = a.small[i];
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
        if (lane == 0) pick_write(a, k, o);
    }
}

template <int NW>
static int launch_pick(arsel_ctx *ctx, const PickArgs &a, size_t lds, hipStream_t s)
{
    const int grid = ctx->num_cu * ctx->sched.blocks_per_cu;
    hipLaunchKernelGGL(k_ragged_pick<NW>, dim3(grid), dim3(NW * 64), lds, s, a);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

// Layout of a list buffer for K instances, `items` scan items and `hitems`
// hard chunks: the small, large, hard and easy lists (K ints each), the hard
// instances' first chunks (K), the per-instance least accepted keys (K u64),
// each section 32-byte aligned, then the scan items and the hard chunks.
struct ListLayout {
    int32_t *small, *large, *hard, *easy;
    uint32_t *hc;
    unsigned long long *best;
    RScan *items;
    HItem *hitems;
};

static inline size_t list_ints(int64_t n)
{
    return ((size_t)n + kListAlignInts - 1) / kListAlignInts * kListAlignInts;
}

static inline size_t list_head_ints(int32_t K)
{
    return 7 * list_ints(K);
}

static inline size_t list_bytes(int32_t K, size_t items, size_t hitems)
{
    return list_head_ints(K) * sizeof(int32_t) + items * sizeof(RScan) + hitems * sizeof(HItem);
}

static inline ListLayout list_layout(int32_t *p, int32_t K, size_t items)
{
    const size_t n = list_ints(K);
    ListLayout l;
    l.small = p;
    l.large = p + n;
    l.hard = p + 2 * n;
    l.easy = p + 3 * n;
    l.hc = reinterpret_cast<uint32_t *>(p + 4 * n);
    l.best = reinterpret_cast<unsigned long long *>(p + 5 * n);
    l.items = reinterpret_cast<RScan *>(p + list_head_ints(K));
    l.hitems = reinterpret_cast<HItem *>(l.items + items);
    return l;
}

// Chunk plan of host-built lists: scan items of kScanChunk elements.
constexpr int32_t kHostMaxCh = 1 << 20;

// Chunks per instance on the device path: the item buffer then holds at most
// K (maxch + 1) items, about 2^21 for large K.
static inline int32_t device_maxch(int32_t K)
{
    int64_t m = ((int64_t)1 << 21) / std::max<int32_t>(K, 1);
    return (int32_t)std::min<int64_t>(32, std::max<int64_t>(1, m));
}

// Resident chunk workgroups per compute unit for a piece of `piece` floats.
static int hard_blocks_per_cu(uint32_t piece)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ragged_hard, kHardThreads,
                                                     (size_t)piece * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        n = 1;
    }
    return n < 1 ? 1 : n;
}

// Enqueue scan, split, hard chunks and pick for lists already in place
// (maxch: the hard chunks' plan, at most maxch chunks per instance, which the
// list buffer's chunk capacity must allow).  On a launch failure after the scan
// the accumulators and counters are cleared again, so the next call starts
// from zero.
static int run_ragged(arsel_ctx *ctx, const float *alpha, const int64_t *offsets, int32_t K,
                      const ListLayout &l, int32_t maxch, const uint32_t *n_items_dev,
                      uint32_t n_items_host, const uint32_t *n_large_dev, uint32_t n_large_host,
                      const uint32_t *n_small_dev, uint32_t n_small_host, uint32_t *queue,
                      RAcc *acc, uint64_t seed, uint64_t step, uint32_t t_max, int32_t *index,
                      float *alpha0, uint32_t *trials, hipStream_t s)
{
    const arsel_schedule &sc = ctx->sched;
    const int nw = sc.block_waves;
    const size_t lds = (size_t)nw * sc.wave_max_m * sizeof(float);
    const uint32_t piece = hard_piece(sc.lds_max_m);
    const int scan_grid = ctx->num_cu * kScanBlocksPerCU;
    hipLaunchKernelGGL(k_ragged_scan, dim3(scan_grid), dim3(kScanWaves * 64), 0, s, alpha, offsets,
                       l.items, n_items_dev, n_items_host, acc, queue);
    int rc = hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
    const uint32_t nl = n_large_dev ? (uint32_t)K : n_large_host;
    if (rc == ARSEL_OK && nl > 0) {
        hipLaunchKernelGGL(k_ragged_split, dim3((nl + kSplitThreads - 1) / kSplitThreads), dim3(kSplitThreads), 0, s,
                           offsets, l.large,
                           n_large_dev, n_large_host, acc, maxch, piece, l.hard, l.easy, l.hitems,
                           l.hc, l.best, queue);
        rc = hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
    }
    if (rc == ARSEL_OK) {
        const int grid = ctx->num_cu * hard_blocks_per_cu(piece);
        hipLaunchKernelGGL(k_ragged_hard, dim3(grid), dim3(kHardThreads), (size_t)piece * sizeof(float), s,
                           alpha, offsets, l.hitems, queue, acc, l.best, maxch, piece, seed, step, t_max);
        rc = hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
    }
    if (rc == ARSEL_OK) {
        PickArgs a;
        a.alpha = alpha;
        a.offsets = offsets;
        a.hard = l.hard;
        a.easy = l.easy;
        a.small = l.small;
        a.hitems = l.hitems;
        a.hc = l.hc;
        a.best = l.best;
        a.acc = acc;
        a.n_small_dev = n_small_dev;
        a.n_small_host = n_small_host;
        a.queue = queue;
        a.index = index;
        a.alpha0 = alpha0;
        a.trials = trials;
        a.seed = seed;
        a.step = step;
        a.t_max = t_max;
        a.maxch = maxch;
        a.piece = piece;
        a.wave_max_m = sc.wave_max_m;
        switch (nw) {
        case 4: rc = launch_pick<4>(ctx, a, lds, s); break;
        case 8: rc = launch_pick<8>(ctx, a, lds, s); break;
        case 16: rc = launch_pick<16>(ctx, a, lds, s); break;
        default: rc = ARSEL_ERR_ARG;
        }
    }
    if (rc != ARSEL_OK) {
        (void)hipGetLastError();
        const int64_t n = (int64_t)K * 2;
        hipLaunchKernelGGL(k_ragged_clear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           reinterpret_cast<uint32_t *>(acc), n);
        hipLaunchKernelGGL(k_ragged_reset, dim3(1), dim3(64), 0, s, queue);
        (void)hipGetLastError();
    }
    return rc;
}

// The per-instance accumulators of the context, for K instances (new space
// is cleared on the stream before use).
static int ensure_acc(arsel_ctx *ctx, int32_t K, hipStream_t s)
{
    const size_t need = (size_t)K * sizeof(RAcc);
    if (ctx->inst_bytes >= need) return ARSEL_OK;
    const int rc = ctx_grow(ctx, &ctx->inst, &ctx->inst_bytes, need);
    if (rc) return rc;
    const int64_t n = (int64_t)(ctx->inst_bytes / sizeof(uint32_t));
    hipLaunchKernelGGL(k_ragged_clear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (uint32_t *)ctx->inst, n);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

static int build_lists_on_device(const int64_t *offsets, int32_t K, int32_t wave_max_m,
                                 int32_t maxch, const ListLayout &l, uint32_t *queue, hipStream_t s)
{
    const unsigned grid = (unsigned)(((int64_t)K + kListThreads - 1) / kListThreads);
    hipLaunchKernelGGL(k_list_clear, dim3(1), dim3(512), 0, s, queue);
    if (hipGetLastError() != hipSuccess) return ARSEL_ERR_HIP;
    hipLaunchKernelGGL(k_list_count, dim3(grid), dim3(kListThreads), 0, s, offsets, K, wave_max_m, maxch, queue);
    if (hipGetLastError() != hipSuccess) return ARSEL_ERR_HIP;
    hipLaunchKernelGGL(k_list_scatter, dim3(grid), dim3(kListThreads), 0, s, offsets, K, wave_max_m, maxch,
                       l.small, l.large, l.items, queue);
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

// Scratch of arsel_select_ragged_noalloc: the counters (padded to 256
// bytes), the lists and keys of at most kNoAllocMaxK instances, pools of
// scan items and hard chunks whose share per instance sets the chunk plans
// (so a batch of 10^4 instances is chunked as finely as with the context's
// buffers), and the accumulators, in a file-scope device array (about
// 12.3 MB).  Each GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (ragged_scratch_address).
// Static storage starts zeroed; every launch leaves the accumulators zero and
// the ordering and split kernels set the counters, lists and keys.
constexpr int32_t kNoAllocMaxK = 1 << 16;
constexpr int32_t kNoAllocItemPool = 1 << 18;   // scan items: K (maxch + 1) <= pool + K
constexpr int32_t kNoAllocHardPool = 1 << 16;   // hard chunks: K hard_maxch <= pool
constexpr size_t kNoAllocItems = (size_t)kNoAllocItemPool + kNoAllocMaxK;
constexpr size_t kNoAllocHItems = (size_t)kNoAllocHardPool;
constexpr size_t kScratchQueueWords = 512;   // the queue words, 2 KB
static_assert(kQueueWordsAll <= (int)kScratchQueueWords && kQueueWordsAll * 4 <= (int)kQueueBytes, "queue words");
constexpr size_t kScratchListWords = 7 * (size_t)kNoAllocMaxK + sizeof(RScan) / 4 * kNoAllocItems +
                                     sizeof(HItem) / 4 * kNoAllocHItems;
constexpr size_t kScratchWords = kScratchQueueWords + kScratchListWords + 2 * (size_t)kNoAllocMaxK;
static __device__ __align__(256) uint32_t scratch[kScratchWords];

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

static int ragged_checks(arsel_ctx *ctx)
{
    const arsel_schedule &sc = ctx->sched;
    const size_t lds = std::max<size_t>((size_t)hard_piece(sc.lds_max_m), (size_t)sc.block_waves * sc.wave_max_m) *
                       sizeof(float);
    return lds > ctx->lds_per_block - 2048 ? ARSEL_ERR_ARG : ARSEL_OK;
}

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
    if ((rc = ragged_checks(ctx))) return rc;
    const arsel_schedule &sc = ctx->sched;
    hipStream_t s = (hipStream_t)stream;
    // Under graph capture the lists are built on the device, inside the graph,
    // in their own buffer: a replay then depends on no list a later call
    // leaves in the context.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) return ARSEL_ERR_HIP;
    if (cap != hipStreamCaptureStatusNone) host_sizes = nullptr;
    if ((rc = ensure_acc(ctx, K, s))) return rc;
    RAcc *acc = (RAcc *)ctx->inst;

    if (host_sizes) {
        // The lists depend only on the sizes and the split (positions are
        // relative to offsets[0]): a call with those of the lists already on
        // the device reuses them.
        const bool same = ctx->order_split == sc.wave_max_m && ctx->order_sizes.size() == (size_t)K &&
                          std::equal(host_sizes, host_sizes + K, ctx->order_sizes.begin());
        if (!same) {
            ctx->order_split = -1;
            // Longest first within each list (counting sort on floor(log2 M),
            // O(K)); the lists go to the device through a pinned staging
            // buffer (reused once the previous copy has finished).
            const int32_t maxch = kHostMaxCh;
            size_t nb_s[64] = {}, nb_l[64] = {}, nb_i[64] = {};
            size_t n_items = 0, n_large = 0, n_small = 0;
            int64_t off = 0;
            for (int32_t k = 0; k < K; ++k) {
                const int64_t m = host_sizes[k];
                const int c = size_class(m);
                if (m <= sc.wave_max_m || bad_size(m)) {
                    ++nb_s[c];
                    ++n_small;
                } else {
                    const size_t n = (size_t)chunk_plan(off, m, maxch).nch;
                    ++nb_l[c];
                    ++n_large;
                    nb_i[c] += n;
                    n_items += n;
                }
                if (!bad_size(m)) off += m;
            }
            const size_t bytes = list_bytes(K, n_items, n_items);
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
            const int32_t *held = ctx->order;
            rc = ctx_grow(ctx, (void **)&ctx->order, &ctx->order_bytes, bytes);
            if (rc || ctx->order != held) ctx->order_split = -1;
            if (rc) return rc;
            size_t ps[64], pl[64], pi[64];
            size_t rs = 0, rl = 0, ri = 0;
            for (int b = 63; b >= 0; --b) {
                ps[b] = rs;
                rs += nb_s[b];
                pl[b] = rl;
                rl += nb_l[b];
                pi[b] = ri;
                ri += nb_i[b];
            }
            const ListLayout h = list_layout(ctx->staging, K, n_items);
            off = 0;
            for (int32_t k = 0; k < K; ++k) {
                const int64_t m = host_sizes[k];
                const int c = size_class(m);
                if (m <= sc.wave_max_m || bad_size(m)) {
                    h.small[ps[c]++] = k;
                } else {
                    h.large[pl[c]++] = k;
                    const ChunkPlan p = chunk_plan(off, m, maxch);
                    for (int32_t ch = 0; ch < p.nch; ++ch) h.items[pi[c]++] = chunk_item(p, off, m, k, ch);
                }
                if (!bad_size(m)) off += m;
            }
            // the hard chunks are written on the device: copy up to the scan items' end
            const size_t copy = bytes - n_items * sizeof(HItem);
            if (hipMemcpyAsync(ctx->order, ctx->staging, copy, hipMemcpyHostToDevice, s) != hipSuccess)
                return ARSEL_ERR_HIP;
            if (!ctx->staging_event && hipEventCreateWithFlags(&ctx->staging_event, hipEventDisableTiming) != hipSuccess)
                return ARSEL_ERR_HIP;
            if (hipEventRecord(ctx->staging_event, s) != hipSuccess) return ARSEL_ERR_HIP;
            ctx->order_items = (uint32_t)n_items;
            ctx->order_large = (uint32_t)n_large;
            ctx->order_waves = (uint32_t)n_small;
            try {
                ctx->order_sizes.assign(host_sizes, host_sizes + K);
                ctx->order_split = sc.wave_max_m;
            } catch (...) {
                ctx->order_sizes.clear();   // the lists stay valid for this call only
            }
        }
        return run_ragged(ctx, alpha, offsets, K, list_layout(ctx->order, K, ctx->order_items),
                          kHostMaxCh, nullptr, ctx->order_items, nullptr, ctx->order_large, nullptr, ctx->order_waves,
                          ctx->queue, acc, seed, step, t_max, index, alpha0, trials, s);
    }
    const int32_t maxch = device_maxch(K);
    if ((rc = ctx_grow(ctx, (void **)&ctx->order_dev, &ctx->order_dev_bytes,
                       list_bytes(K, (size_t)K * (maxch + 1), (size_t)K * maxch))))
        return rc;
    const ListLayout l = list_layout(ctx->order_dev, K, (size_t)K * (maxch + 1));
    if ((rc = build_lists_on_device(offsets, K, sc.wave_max_m, maxch, l, ctx->queue, s))) return rc;
    return run_ragged(ctx, alpha, offsets, K, l, maxch, ctx->queue + kQNItems, 0, ctx->queue + kQNLarge, 0,
                      ctx->queue + kQNSmall, 0, ctx->queue, acc, seed, step, t_max, index, alpha0,
                      trials, s);
}

// The same selection with every list and counter in the GPU's static scratch
// array: no allocation of any kind.  The ordering kernel sets every counter
// before the other kernels read them, and every launch leaves the
// accumulators zero, so nothing an earlier call left in the array is read.
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
    if ((rc = ragged_checks(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    uint32_t *queue = static_cast<uint32_t *>(ctx->scratch);
    int32_t *lists = reinterpret_cast<int32_t *>(queue + kScratchQueueWords);
    RAcc *acc = reinterpret_cast<RAcc *>(queue + kScratchQueueWords + kScratchListWords);
    const ListLayout l = list_layout(lists, K, kNoAllocItems);
    const int32_t maxch = std::min<int32_t>(32, kNoAllocItemPool / K);
    const int32_t hard_maxch = std::min<int32_t>(32, kNoAllocHardPool / K);
    if ((rc = build_lists_on_device(offsets, K, ctx->sched.wave_max_m, maxch, l, queue, s))) return rc;
    return run_ragged(ctx, alpha, offsets, K, l, hard_maxch, queue + kQNItems, 0, queue + kQNLarge, 0,
                      queue + kQNSmall, 0, queue, acc, seed, step, t_max, index, alpha0, trials, s);
}
