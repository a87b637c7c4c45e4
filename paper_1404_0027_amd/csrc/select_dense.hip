// Dense batched selection: K instances of M reactions, AoS / SoA / broadcast.
//
// The paper runs one thread block per realization and one thread per
// reaction (section "Results / Implementation").  Here a workgroup owns a
// tile of TK instances: it streams the tile's propensities from HBM with
// coalesced loads (SoA: TK consecutive instances per row, 16-byte loads),
// transposes them into LDS so that each instance is contiguous, and then
// each wavefront selects for one instance at a time, gathering candidates
// from LDS.  When a tile does not fit in LDS, each wavefront reads its
// instance straight from global memory.
#include "select_core.hpp"
#include "launch.hpp"

namespace arsel {

struct DenseArgs {
    const float *alpha;
    int64_t ld;
    const float *bound;
    int32_t *index;
    float *alpha0;
    uint32_t *trials;
    uint64_t seed, step;
    int32_t M, K;
    int32_t tk;        // instances per tile
    int32_t mp;        // LDS row stride (floats)
    uint32_t t_max;
    uint32_t flags;
    int32_t layout;    // 0 AoS (ld == 0: broadcast), 1 SoA
    int32_t vec4;      // SoA tiles may use 16-byte loads
};

__device__ __forceinline__ void write_outcome(const DenseArgs &a, int k, const Outcome &o)
{
    if (lane_id() == 0) {
        a.index[k] = o.index;
        if (a.alpha0) a.alpha0[k] = o.alpha0;
        if (a.trials) a.trials[k] = o.trials;
    }
}

constexpr int kMaxTile = 64;     // instances per tile (upper bound)
constexpr int kBatch = 6;        // loads issued per thread before their LDS stores

// Running maximum of the raw bits of non-negative floats: for finite x >= 0
// the float order is the unsigned order of the bits, and every negative,
// +inf or NaN has bits >= 0x7F800000.  A maximum below 0x7F800000 therefore
// certifies a valid vector and IS the bits of alpha_max; anything else (an
// invalid entry, or a harmless -0.0) sends the instance to the exact scan.
__device__ __forceinline__ uint32_t umax4(uint32_t m, f32x4 v)
{
    m = max(m, __float_as_uint(v.x));
    m = max(m, __float_as_uint(v.y));
    m = max(m, __float_as_uint(v.z));
    return max(m, __float_as_uint(v.w));
}

constexpr uint32_t kInvalidBits = 0x7F800000u;

// Copy the tile into LDS: instance t of the tile becomes lds[t*mp .. t*mp+M).
// Each thread issues kBatch loads before storing any of them, and calls
// mid() between issuing and storing the first batch, so that work which does
// not depend on the propensities runs while the loads are in flight.  The
// SoA path also returns, per thread, the bit-maximum of the 4 instances it
// touched (instances 4*(tid % qpr) .. +3); other paths return false.
template <int NW, class Mid>
__device__ __forceinline__ bool stage_tile(const DenseArgs &a, float *lds, int k0, int nk,
                                           bool bcast, uint32_t mx[4], Mid &&mid)
{
    const int tid = threadIdx.x;
    constexpr int NT = NW * 64;
    const int M = a.M;
    if (a.layout == 1 && a.vec4 && nk == a.tk && !bcast) {
        // SoA, full aligned tile: a lane reads 4 consecutive instances of one row.
        const int qpr = a.tk >> 2;
        const int qshift = __builtin_ctz(qpr);
        const int total = M * qpr;                         // float4 slots in the tile
        const int row_step = NT >> qshift;                 // rows advanced per slot
        const int j0 = tid >> qshift, q = tid & (qpr - 1);
        const float *src = a.alpha + k0 + 4 * q;
        float *dst0 = lds + (4 * q) * a.mp;
        mx[0] = mx[1] = mx[2] = mx[3] = 0;
        f32x4 v[kBatch];
        auto issue = [&](int base) {
#pragma unroll
            for (int u = 0; u < kBatch; ++u)
                if (base + u * NT + tid < total)
                    v[u] = load_stream4(src + (int64_t)(j0 + ((base >> qshift) + u * row_step)) * a.ld);
        };
        auto store = [&](int base) {
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (base + u * NT + tid < total) {
                    float *d = dst0 + j0 + (base >> qshift) + u * row_step;
                    d[0] = v[u].x;
                    d[a.mp] = v[u].y;
                    d[2 * a.mp] = v[u].z;
                    d[3 * a.mp] = v[u].w;
                    mx[0] = max(mx[0], __float_as_uint(v[u].x));
                    mx[1] = max(mx[1], __float_as_uint(v[u].y));
                    mx[2] = max(mx[2], __float_as_uint(v[u].z));
                    mx[3] = max(mx[3], __float_as_uint(v[u].w));
                }
            }
        };
        issue(0);
        mid();
        store(0);
        for (int base = kBatch * NT; base < total; base += kBatch * NT) {
            issue(base);
            store(base);
        }
        return true;
    }
    mid();
    if (bcast) {
        for (int j = tid; j < M; j += NT) lds[j] = a.alpha[j];
        return false;
    }
    if (a.layout == 0 && a.ld == a.M) {
        // AoS with contiguous rows: the tile is one contiguous span of nk*M floats.
        const float *src = a.alpha + (int64_t)k0 * M;
        const int total = nk * M;
        const int head = (int)(((16 - ((uintptr_t)src & 15)) & 15) >> 2);   // floats to 16 B
        const int h = head < total ? head : total;
        if (tid < h) lds[tid] = src[tid];
        const int nq = (total - h) >> 2;
        const float *src4 = src + h;
        for (int base = 0; base < nq; base += kBatch * NT) {
            f32x4 v[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int i = base + u * NT + tid;
                if (i < nq) v[u] = load_stream4(src4 + 4 * i);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int i = base + u * NT + tid;
                if (i < nq) {
                    float *dst = lds + h + 4 * i;
                    dst[0] = v[u].x;
                    dst[1] = v[u].y;
                    dst[2] = v[u].z;
                    dst[3] = v[u].w;
                }
            }
        }
        for (int f = h + 4 * nq + tid; f < total; f += NT) lds[f] = src[f];
        return false;
    }
    if (a.layout == 0) {
        // AoS with padded rows: row by row.
        for (int t = 0; t < nk; ++t)
            for (int j = tid; j < M; j += NT)
                lds[t * a.mp + j] = a.alpha[(int64_t)(k0 + t) * a.ld + j];
        return false;
    }
    // SoA, partial or unaligned tile.
    const int total = M * nk;
    for (int i = tid; i < total; i += NT) {
        const int j = i / nk;
        const int c = i - j * nk;
        lds[c * a.mp + j] = a.alpha[(int64_t)j * a.ld + k0 + c];
    }
    return false;
}

// Rounds whose random draws are computed while the tile streams in.
constexpr int kPreRounds = 4;
constexpr uint32_t kNoCand = 0xFFFFFFFFu;

// The two trials of one lane in one round: candidates (kNoCand when the
// Lemire draw rejects or the trial is beyond t_max) and u words.
struct LaneDraw {
    uint32_t ja, ua, jb, ub;
};

__device__ __forceinline__ LaneDraw lane_draw(const Stream &st, uint32_t r, uint32_t M,
                                              uint32_t thresh, uint32_t t_max)
{
    const int lane = lane_id();
    const uint64_t t0 = (uint64_t)r * kRoundTrials;
    const Words w = st.block((uint32_t)(t0 >> 1) + (uint32_t)lane);
    const uint64_t ta = t0 + 2 * (uint64_t)lane;
    LaneDraw d;
    uint32_t j;
    d.ja = (lemire(w.w0, M, thresh, j) && ta < t_max) ? j : kNoCand;
    d.ua = w.w1;
    d.jb = (lemire(w.w2, M, thresh, j) && ta + 1 < t_max) ? j : kNoCand;
    d.ub = w.w3;
    return d;
}

// The candidates' propensities of one round (both gathers issued together;
// a rejected draw reads entry 0, whose value is then ignored).
struct RoundVals {
    float a, b;
};

template <class Acc>
__device__ __forceinline__ RoundVals gather_round(const Acc &A, const LaneDraw &d)
{
    return {A(d.ja != kNoCand ? d.ja : 0u), A(d.jb != kNoCand ? d.jb : 0u)};
}

// Decide one round from its draws and gathered values: least accepted
// (trial << 32 | j) or kNoAccept.  envs is the envelope times 2^-32 (exact),
// so w * envs is the real number u * env rounded once, as fl64(u * env) with
// u = w 2^-32.
__device__ __forceinline__ uint64_t decide_round(const LaneDraw &d, RoundVals x, double envs,
                                                 uint32_t r)
{
    const bool acca = (d.ja != kNoCand) & ((double)d.ua * envs < (double)x.a);
    const bool accb = (d.jb != kNoCand) & ((double)d.ub * envs < (double)x.b);
    const uint64_t ma = __ballot(acca), mb = __ballot(accb);
    if ((ma | mb) == 0) return kNoAccept;
    const uint64_t t0 = (uint64_t)r * kRoundTrials;
    const int la = first_lane(ma), lb = first_lane(mb);
    if (la <= lb) return ((t0 + 2 * (uint64_t)la) << 32) | readlane_u32(d.ja, la);
    return ((t0 + 2 * (uint64_t)lb + 1) << 32) | readlane_u32(d.jb, lb);
}

template <class Acc>
__device__ __forceinline__ uint64_t resolve_round(const Acc &A, const LaneDraw &d, double envs,
                                                  uint32_t r)
{
    return decide_round(d, gather_round(A, d), envs, r);
}

// Envelope scaled by 2^-32 for decide_round (exact in binary64).
__device__ __forceinline__ double scaled_env(float env)
{
    return (double)env * 0x1p-32;
}

// Row stride of the partial maxima (one word more than the 64 slots, so that
// a wavefront reading one instance's slots touches 64 different banks).
constexpr int kPartStride = 65;

// Per-instance state of a tile.
struct TileState {
    uint64_t best[kMaxTile];      // least accepted (trial << 32 | j) so far
    uint64_t open;                // instances whose rounds are still handed out
    uint32_t next[kMaxTile];      // next round to hand out
    double env[kMaxTile];         // envelope times 2^-32 (scaled_env)
    float amax[kMaxTile];
    float alpha0[kMaxTile];
    int32_t index[kMaxTile];      // 0 in the trial phase, < 0 decided status
    int32_t written[kMaxTile];    // outcome already stored
};

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_select_tile(DenseArgs a)
{
    extern __shared__ float lds[];
    __shared__ TileState ts;
    // per-(wave, row of 16 lanes) partial bit-maxima of each instance, after the tile
    uint32_t *part = reinterpret_cast<uint32_t *>(lds + (size_t)a.tk * a.mp);
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = lane_id();
    const int k0 = xcd_tile(blockIdx.x, gridDim.x) * a.tk;
    const int nk = min(a.tk, a.K - k0);
    const uint32_t M = (uint32_t)a.M;
    const bool bcast = (a.layout == 0 && a.ld == 0);
    const bool want_a0 = a.alpha0 != nullptr;
    const uint32_t rounds = (uint32_t)(((uint64_t)a.t_max + kRoundTrials - 1) / kRoundTrials);
    const bool own = wave < nk;
    const Stream st_own = make_stream(a.seed, a.step, (uint32_t)(k0 + wave), kTagUniform);

    // Stage the tile; meanwhile draw the first rounds of this wave's instance.
    uint32_t thresh = 0;
    LaneDraw pre[kPreRounds];
    uint32_t mx[4];
    auto mid = [&]() {
        thresh = lemire_threshold(M);
#pragma unroll
        for (int r = 0; r < kPreRounds; ++r)
            pre[r] = (own && (uint32_t)r < rounds) ? lane_draw(st_own, r, M, thresh, a.t_max)
                                                   : LaneDraw{kNoCand, 0u, kNoCand, 0u};
    };
    const bool fused = stage_tile<NW>(a, lds, k0, nk, bcast, mx, mid);
    if (fused) {
        // reduce over the lanes of a row that share instances (same lane % qpr)
        const int qpr = a.tk >> 2;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            uint32_t x = mx[c];
            if (qpr <= 1) x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x121, 0xF, 0xF, false));
            if (qpr <= 2) x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x122, 0xF, 0xF, false));
            if (qpr <= 4) x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x124, 0xF, 0xF, false));
            if (qpr <= 8) x = max(x, (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x128, 0xF, 0xF, false));
            mx[c] = x;
        }
        const int rl = lane & 15;
        if (rl < qpr) {
            const int slot = wave * 4 + (lane >> 4);
#pragma unroll
            for (int c = 0; c < 4; ++c) part[(4 * rl + c) * kPartStride + slot] = mx[c];
        }
    }
    if (tid == 0) ts.open = 0;
    __syncthreads();

    // Each wave decides its instances and runs their first rounds.
    for (int t = wave; t < nk; t += NW) {
        const int k = k0 + t;
        const ContigAcc acc{lds + (bcast ? 0 : t * a.mp)};
        const float *bk = a.bound ? a.bound + k : nullptr;
        // the candidates of the pre-drawn rounds do not depend on the
        // envelope: gather them all before the maximum is reduced
        RoundVals pv[kPreRounds];
        if (t == wave) {
#pragma unroll
            for (int rr = 0; rr < kPreRounds; ++rr) pv[rr] = gather_round(acc, pre[rr]);
        }
        ScanState sc;
        uint32_t mb = 0;
        if (fused) mb = wave_max_u32(lane < NW * 4 ? part[t * kPartStride + lane] : 0u);
        if (fused && mb < kInvalidBits && !bk) {
            // certified valid: alpha_max from the fused maximum
            sc.scanned = true;
            sc.amax = __uint_as_float(mb);
            sc.decided = decide_status(true, false, sc.amax, nullptr, a.flags, sc.env, sc.o);
            if (!sc.decided && want_a0) {
                const int shift = 63 - ceil_log2_u32(M) - exponent_above(sc.amax);
                sc.o.alpha0 = fixed_to_float(wave_fixed_sum(acc, M, shift), shift);
            }
        } else {
            sc = wave_prepare(acc, M, bk, a.flags, want_a0);
        }
        uint64_t key = kNoAccept;
        uint32_t r = 0;
        if (!sc.decided) {
            const double envs = scaled_env(sc.env);
            // instances beyond the first NW of a tile start at round 0 in the
            // batches below
            if (t == wave) {
#pragma unroll
                for (int rr = 0; rr < kPreRounds; ++rr) {
                    if ((uint32_t)rr < rounds && key == kNoAccept) {
                        key = decide_round(pre[rr], pv[rr], envs, rr);
                        r = rr + 1;
                    }
                }
            }
        }
        if (sc.decided || key != kNoAccept) {
            // resolved: write now, off the workgroup's critical path
            Outcome o = sc.o;
            if (!sc.decided) {
                o.index = (int32_t)(uint32_t)key;
                o.trials = (uint32_t)(key >> 32) + 1;
            }
            write_outcome(a, k, o);
        }
        if (lane == 0) {
            ts.index[t] = sc.decided ? sc.o.index : 0;
            ts.written[t] = (sc.decided || key != kNoAccept) ? 1 : 0;
            ts.alpha0[t] = sc.o.alpha0;
            ts.amax[t] = sc.amax;
            ts.env[t] = scaled_env(sc.env);
            ts.best[t] = key;
            ts.next[t] = r;
            if (!sc.decided && key == kNoAccept && r < rounds)
                atomicOr((unsigned long long *)&ts.open, 1ull << t);
        }
    }
    __syncthreads();

    // Remaining rounds, in batches: the open instances (at most NW per batch)
    // share the NW waves round-robin, instance i of the batch running rounds
    // next .. next + n_i - 1 at once.  A barrier ends the batch; an instance
    // whose batch accepted closes with the least accepted trial (every lower
    // round was run in an earlier batch and rejected), so the result is the
    // sequential rule's.
    for (;;) {
        const uint64_t open = uniform_u64(ts.open);
        if (open == 0) break;
        const int cnt = __popcll(open);
        const int slots = cnt < NW ? cnt : NW;
        const int i = wave % slots;
        uint64_t m = open;
        for (int c = 0; c < i; ++c) m &= m - 1;
        const int t = (int)__builtin_ctzll(m);
        const uint32_t base = uniform_u32(ts.next[t]);
        const uint32_t r = base + (uint32_t)(wave / slots);
        if (r < rounds) {
            const Stream st = make_stream(a.seed, a.step, (uint32_t)(k0 + t), kTagUniform);
            const ContigAcc acc{lds + (bcast ? 0 : t * a.mp)};
            const uint64_t key = resolve_round(acc, lane_draw(st, r, M, thresh, a.t_max), ts.env[t], r);
            if (key != kNoAccept && lane == 0)
                atomicMin((unsigned long long *)&ts.best[t], (unsigned long long)key);
        }
        __syncthreads();
        if (wave == i && lane == 0) {
            const uint32_t n = (uint32_t)((NW - i + slots - 1) / slots);
            ts.next[t] = base + n;
            if (ts.best[t] != kNoAccept || base + n >= rounds)
                atomicAnd((unsigned long long *)&ts.open, ~(1ull << t));
        }
        __syncthreads();
    }

    // Finish: fallback where every round rejected, then write.
    for (int tt = wave; tt < nk; tt += NW) {
        const int k = k0 + tt;
        if (ts.written[tt]) continue;
        Outcome o;
        o.alpha0 = ts.alpha0[tt];
        if (ts.index[tt] < 0) {
            o.index = ts.index[tt];
            o.trials = 0;
        } else if (ts.best[tt] != kNoAccept) {
            o.index = (int32_t)(uint32_t)ts.best[tt];
            o.trials = (uint32_t)(ts.best[tt] >> 32) + 1;
        } else {
            const Stream st = make_stream(a.seed, a.step, (uint32_t)k, kTagUniform);
            const ContigAcc acc{lds + (bcast ? 0 : tt * a.mp)};
            const bool scanned = (a.bound == nullptr) || (a.flags & kDebugCheckBound) || want_a0;
            o = wave_fallback(acc, M, scanned, ts.amax[tt], st, a.t_max, ts.alpha0[tt]);
        }
        write_outcome(a, k, o);
    }
}

// Large M: one wavefront per instance, gathers from global memory.
template <int NW>
__global__ __launch_bounds__(NW * 64) void k_select_global(DenseArgs a)
{
    const int k = blockIdx.x * NW + (threadIdx.x >> 6);
    if (k >= a.K) return;
    StridedAcc acc;
    if (a.layout == 0) {
        acc.p = a.alpha + (int64_t)k * a.ld;
        acc.stride = 1;
    } else {
        acc.p = a.alpha + k;
        acc.stride = a.ld;
    }
    const Stream st = make_stream(a.seed, a.step, (uint32_t)k, kTagUniform);
    const Outcome o = wave_select(acc, (uint32_t)a.M, a.bound ? a.bound + k : nullptr, a.flags, st,
                                  a.t_max, a.alpha0 != nullptr);
    write_outcome(a, k, o);
}

int launch_tile(arsel_ctx *ctx, const DenseArgs &a, int grid, size_t lds, hipStream_t s)
{
    // Automatic choice (no explicit configuration): a launch of about one
    // tile per CU finishes sooner with 16 wavefronts sharing each tile's
    // rounds; with several tiles per CU, 8 wavefronts per tile let two tiles
    // overlap on a CU (measured: 1.54 vs 1.26 TB/s at 256 tiles, 2.73 vs 2.32
    // at 4096 tiles, 3.12 vs 2.51 at 62500 tiles).
    int waves = ctx->dense_waves;
    if (waves == 0) waves = grid <= ctx->num_cu ? 16 : 8;
    switch (waves) {
    case 4:
        hipLaunchKernelGGL(k_select_tile<4>, dim3(grid), dim3(256), lds, s, a);
        break;
    case 8:
        hipLaunchKernelGGL(k_select_tile<8>, dim3(grid), dim3(512), lds, s, a);
        break;
    default:
        hipLaunchKernelGGL(k_select_tile<16>, dim3(grid), dim3(1024), lds, s, a);
        break;
    }
    return hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
}

}  // namespace arsel

using namespace arsel;

extern "C" int arsel_select(arsel_ctx *ctx, const float *alpha, int32_t M, int32_t K, int64_t ld,
                            int layout, const float *bound, uint64_t seed, uint64_t step,
                            uint32_t t_max, uint32_t flags, int32_t *index, float *alpha0,
                            uint32_t *trials, void *stream)
{
    if (!ctx) return ARSEL_ERR_NULL;
    if (M < 1 || K < 0) return ARSEL_ERR_SIZE;
    if (layout != ARSEL_AOS && layout != ARSEL_SOA) return ARSEL_ERR_LAYOUT;
    if (layout == ARSEL_AOS && ld != 0 && ld < M) return ARSEL_ERR_LD;
    if (layout == ARSEL_SOA && ld < K) return ARSEL_ERR_LD;
    if (K == 0) return ARSEL_OK;
    if (!alpha || !index) return ARSEL_ERR_NULL;
    int rc = ctx_activate(ctx);
    if (rc) return rc;

    DenseArgs a;
    a.alpha = alpha;
    a.ld = ld;
    a.bound = bound;
    a.index = index;
    a.alpha0 = alpha0;
    a.trials = trials;
    a.seed = seed;
    a.step = step;
    a.M = M;
    a.K = K;
    a.t_max = t_max;
    a.flags = flags;
    a.layout = layout;
    a.mp = M;
    a.vec4 = 0;
    hipStream_t s = (hipStream_t)stream;

    const bool bcast = (layout == ARSEL_AOS && ld == 0);
    // one vector for every instance: packed rounds (any trial width gives the
    // same answer; the bound and debug modes keep the tile kernel)
    if (bcast && bound == nullptr && packed_lds_bytes(M, false) + 4096 <= ctx->lds_per_block)
        return launch_packed(ctx, alpha, nullptr, M, K, seed, step, t_max, index, alpha0, trials, s);
    const size_t row = (size_t)M * sizeof(float);
    const size_t budget = ctx->tile_lds_bytes;
    int tk = bcast ? ctx->dense_tile : (int)std::min<size_t>((size_t)ctx->dense_tile, budget / row);
    if (bcast && row > budget) tk = 0;
    if (tk >= 1) {
        if (layout == ARSEL_SOA) {
            // power-of-two tiles of >= 4 instances allow 16-byte loads
            int p = 1;
            while (p * 2 <= tk) p *= 2;
            tk = p;
            a.vec4 = (tk >= 4 && (ld % 4) == 0 && ((uintptr_t)alpha % 16) == 0) ? 1 : 0;
        }
        a.tk = tk;
        const size_t lds = (bcast ? 1 : (size_t)tk) * (size_t)a.mp * sizeof(float) +
                           (size_t)tk * kPartStride * sizeof(uint32_t);   // partial maxima: up to 64 slots per instance
        const int grid = (K + tk - 1) / tk;
        rc = launch_tile(ctx, a, grid, lds, s);
    } else {
        a.tk = 1;
        const int nw = 4;
        const int grid = (K + nw - 1) / nw;
        hipLaunchKernelGGL(k_select_global<4>, dim3(grid), dim3(nw * 64), 0, s, a);
        rc = hipGetLastError() == hipSuccess ? ARSEL_OK : ARSEL_ERR_HIP;
    }
    return rc;
}

