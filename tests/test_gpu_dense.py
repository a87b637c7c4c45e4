"""GPU parity of arsel_select (dense batches) against the CPU oracle:
bit-exact indices, trial counts and fixed-point alpha_0."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_0027_amd import arsel, workloads
from tests.parity import assert_same, dense_both

pytestmark = pytest.mark.gpu

AOS, SOA = arsel.AOS, arsel.SOA


def test_uniform_vector_broadcast(gpu):
    """M=16 U(0,1], one vector for K=1024 instances, Philox seed 1."""
    a = workloads.uniform_vector(16, seed=1)
    for step in (0, 1, 2, 999, 2**32 + 5):
        g, o = dense_both(a, 16, 1024, 0, AOS, seed=1, step=step)
        assert_same(g, o, f"broadcast step {step}")


def test_lognormal_soa_full_size(gpu):
    """R=4096 realizations x M=1029 SoA, lognormal(0,2) with 30% zeros."""
    buf = workloads.lognormal_soa(M=1029, K=4096, seed=2, buffers=2)
    for b, step in ((0, 0), (1, 1), (0, 999)):
        g, o = dense_both(buf[b], 1029, 4096, 4096, SOA, seed=1, step=step)
        assert_same(g, o, f"soa buffer {b} step {step}")


@pytest.mark.parametrize("K,ld", [(4100, 4104), (4100, 4103), (3, 3), (37, 40), (1, 1)])
def test_soa_tails_and_alignment(gpu, K, ld):
    rng = np.random.default_rng(K + ld)
    M = 1029
    a = np.zeros((M, ld), np.float32)
    a[:, :K] = rng.lognormal(0, 2, size=(M, K)).astype(np.float32)
    a[:, :K][rng.random((M, K)) < 0.3] = 0
    g, o = dense_both(a, M, K, ld, SOA, seed=5, step=3)
    assert_same(g, o, f"soa K={K} ld={ld}")


@pytest.mark.parametrize("M,K,ld", [(1029, 300, 1031), (1029, 4096, 1029), (5000, 37, 5000),
                                    (64, 1000, 64), (1, 50, 1), (2, 70, 3)])
def test_aos(gpu, M, K, ld):
    rng = np.random.default_rng(M * 7 + K)
    a = rng.exponential(1.0, size=(K, ld)).astype(np.float32)
    a[rng.random((K, ld)) < 0.2] = 0
    g, o = dense_both(a, M, K, ld, AOS, seed=11, step=7)
    assert_same(g, o, f"aos M={M} K={K} ld={ld}")


@pytest.mark.parametrize("layout", [AOS, SOA])
def test_large_m_global_path(gpu, layout):
    """M too large for an LDS tile: one wavefront per instance reads global memory."""
    rng = np.random.default_rng(3)
    M, K = 30000, 24
    a = rng.lognormal(0, 3, size=(K, M)).astype(np.float32)
    if layout == SOA:
        a = np.ascontiguousarray(a.T)
        ld = K
    else:
        ld = M
    g, o = dense_both(a, M, K, ld, layout, seed=2, step=8)
    assert_same(g, o, f"global layout {layout}")


def test_very_large_m(gpu):
    """Two instances of 2^24 + 7 reactions (lognormal(0, 3), AoS): indices above
    2^24 (beyond float precision), L = 25 in the fixed-point scale, and a
    fallback prefix over 16.8 million weights; t_max 4096 and 0."""
    rng = np.random.default_rng(21)
    M, K = (1 << 24) + 7, 2
    a = rng.lognormal(0, 3, size=(K, M)).astype(np.float32)
    for t_max in (4096, 0):
        g, o = dense_both(a, M, K, M, AOS, seed=5, step=t_max, t_max=t_max)
        assert_same(g, o, f"M=2^24+7 t_max={t_max}")
    assert np.all(g[0] >= 0)


@pytest.mark.parametrize("t_max", [0, 1, 2, 3, 63, 127, 128, 129, 255, 4096])
def test_trial_budgets_and_fallback(gpu, t_max):
    """Budgets that end inside a round, and forced fallbacks (t_max = 0)."""
    rng = np.random.default_rng(t_max)
    M, K = 777, 512
    a = rng.lognormal(0, 3, size=(K, M)).astype(np.float32)
    a[rng.random((K, M)) < 0.3] = 0
    g, o = dense_both(a, M, K, M, AOS, seed=9, step=t_max, t_max=t_max)
    assert_same(g, o, f"t_max {t_max}")
    if t_max <= 3:
        assert np.any(g[2] == t_max + 1)    # the fallback fired somewhere


def test_supplied_bounds(gpu):
    rng = np.random.default_rng(4)
    M, K = 300, 256
    a = rng.random((K, M)).astype(np.float32)
    amax = a.max(axis=1)
    for bound, flags in ((amax * 2, 0), (amax.copy(), 0), (amax * 1000, 0),
                         (amax / 2, arsel.DEBUG_CHECK_BOUND), (amax * 3, arsel.DEBUG_CHECK_BOUND)):
        g, o = dense_both(a, M, K, M, AOS, seed=3, step=1, bound=bound.astype(np.float32),
                          flags=flags)
        assert_same(g, o, f"bound flags={flags}")
    special = np.array([0, -1, np.nan, np.inf] * 64, np.float32)
    g, o = dense_both(a, M, K, M, AOS, seed=3, step=1, bound=special)
    assert_same(g, o, "special bounds")
    assert set(np.unique(g[0])) == {-1, -2}


def test_edge_rows(gpu):
    """All-zero, invalid, subnormal, single-nonzero, near-FLT_MAX and -0.0 rows."""
    M = 200
    rows = []
    rows.append(np.zeros(M))                                         # -1
    r = np.ones(M); r[17] = np.nan; rows.append(r)                   # -2
    r = np.ones(M); r[0] = -1.0; rows.append(r)                      # -2
    r = np.ones(M); r[199] = np.inf; rows.append(r)                  # -2
    r = np.zeros(M); r[5] = 1e-3; rows.append(r)                     # single nonzero
    rows.append(np.full(M, 3e-44))                                   # subnormal
    r = np.full(M, 1e-45); r[::3] = 7e-45; rows.append(r)            # subnormal mix
    r = np.full(M, 3.0e38); r[::2] = 1.0; rows.append(r)             # near FLT_MAX (alpha_0 = inf)
    r = np.full(M, -0.0); r[42] = 2.0; rows.append(r)                # negative zeros
    r = np.geomspace(1e-30, 1e30, M); rows.append(r)                 # 60 decades
    a = np.array(rows, np.float32)
    K = a.shape[0]
    for t_max in (4096, 0, 1):
        g, o = dense_both(a, M, K, M, AOS, seed=21, step=0, t_max=t_max)
        assert_same(g, o, f"edge rows t_max={t_max}")
    assert g[0][0] == -1 and list(g[0][1:4]) == [-2, -2, -2] and g[0][4] == 5


@pytest.mark.parametrize("tile,waves", [(1, 4), (4, 4), (8, 8), (16, 16), (32, 16), (64, 16), (5, 8)])
def test_dense_schedule_does_not_change_results(gpu, tile, waves):
    buf = workloads.lognormal_soa(M=1029, K=1024, seed=2)[0]
    ref = dense_both(buf, 1029, 1024, 1024, SOA, seed=1, step=4)[1]
    arsel.set_dense_config(tile, waves)
    try:
        g, _ = dense_both(buf, 1029, 1024, 1024, SOA, seed=1, step=4)
        assert_same(g, ref, f"tile {tile} waves {waves}")
        a = buf.T.copy()
        g, o = dense_both(a, 1029, 1024, 1029, AOS, seed=1, step=4)
        assert_same(g, o, f"aos tile {tile} waves {waves}")
    finally:
        arsel.set_dense_config(0, 0)


def test_host_argument_errors(gpu):
    ctx = arsel.context(0)
    a = torch.ones(100, device=gpu)
    idx = torch.empty(10, dtype=torch.int32, device=gpu)
    st = torch.cuda.current_stream().cuda_stream
    call = lambda M, K, ld, layout, ap=a.data_ptr(), ip=idx.data_ptr(): arsel.select_raw(
        ctx, ap, M, K, ld, layout, None, 1, 0, 4096, 0, ip, None, None, st)
    assert call(10, 10, 9, AOS) == -4       # ld < M
    assert call(10, 10, 9, SOA) == -4       # ld < K
    assert call(10, 10, 10, 7) == -3        # bad layout
    assert call(0, 10, 10, AOS) == -2       # M < 1
    assert call(10, -1, 10, AOS) == -2      # K < 0
    assert call(10, 0, 10, AOS) == 0        # K = 0 is a no-op
    assert call(10, 10, 10, AOS, ap=None) == -1
    with pytest.raises(arsel.ArselError):
        arsel.select(a, 10, 11, 10, AOS, seed=1)   # tensor too small for K*ld


def test_repeatable(gpu):
    buf = workloads.lognormal_soa(M=1029, K=4096, seed=2)[0]
    t = torch.from_numpy(buf).to(gpu)
    r1 = arsel.select(t, 1029, 4096, 4096, SOA, seed=7, step=3)[0].cpu()
    r2 = arsel.select(t, 1029, 4096, 4096, SOA, seed=7, step=3)[0].cpu()
    r3 = arsel.select(t, 1029, 4096, 4096, SOA, seed=7, step=4)[0].cpu()
    assert torch.equal(r1, r2) and not torch.equal(r1, r3)


def test_million_realizations_sampled(gpu):
    """10^6 realizations x M = 1029 (SoA, 4.1 GB) in one launch; 96 sampled
    instances (and the last ones, in the ragged last tile) checked against
    the oracle by instance id."""
    M, K = 1029, 1_000_000
    g = torch.Generator(device="cuda").manual_seed(123)
    a = torch.empty(M, K, device="cuda").log_normal_(0.0, 2.0, generator=g)
    a[torch.rand(M, K, device="cuda", generator=g) < 0.3] = 0.0
    idx, a0, tr = arsel.select(a, M, K, K, arsel.SOA, seed=5, step=2, want_alpha0=True,
                               want_trials=True)
    ids = np.unique(np.r_[np.random.default_rng(0).choice(K, 96, replace=False), K - 3, K - 2, K - 1])
    rows = a[:, torch.from_numpy(ids.astype(np.int64)).cuda()].T.contiguous().cpu().numpy()
    oi, oa, ot = oracle.select_ids(rows, ids.astype(np.uint32), seed=5, step=2, threads=8)
    assert np.array_equal(idx.cpu().numpy()[ids], oi)
    assert np.array_equal(tr.cpu().numpy().view(np.uint32)[ids], ot)
    assert np.array_equal(a0.cpu().numpy()[ids].view(np.uint32), oa.view(np.uint32))


def test_graph_replays_match_eager(gpu):
    """The bench captures its steps in a HIP graph: replays (with eager work
    and synchronisation between them) give the eager results, step by step."""
    M, K, steps = 1029, 4096, 6
    host = workloads.lognormal_soa(M=M, K=K, seed=2, buffers=3)
    bufs = torch.from_numpy(host).cuda()
    out = torch.empty(steps, K, dtype=torch.int32, device="cuda")
    eager = torch.empty_like(out)
    for s in range(steps):
        arsel.select(bufs[s % 3], M, K, K, SOA, seed=1, step=s, index=eager[s])
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap, capture_error_mode="relaxed"):
            for s in range(steps):
                arsel.select(bufs[s % 3], M, K, K, SOA, seed=1, step=s, index=out[s])
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        arsel.select(bufs[0], M, K, K, SOA, seed=9, step=99, index=eager[0].clone())   # eager work between


def test_sensitivity_analysis_shape_sampled(gpu):
    """9 x 1029 x 1000 = 9,261,000 realizations x M = 1029 (SoA, 38 GB) in one
    launch, element offsets far beyond 2^32; sampled instances (and the ragged
    last tile) checked against the oracle by instance id."""
    M, K = 1029, 9 * 1029 * 1000
    g = torch.Generator(device="cuda").manual_seed(321)
    a = torch.empty(M, K, device="cuda")
    for r in range(0, M, 64):
        blk = a[r:r + 64]
        blk.log_normal_(0.0, 2.0, generator=g)
        blk[torch.rand(blk.shape, device="cuda", generator=g) < 0.3] = 0.0
    idx, a0, tr = arsel.select(a, M, K, K, arsel.SOA, seed=9, step=5, want_alpha0=True,
                               want_trials=True)
    ids = np.unique(np.r_[np.random.default_rng(1).choice(K, 64, replace=False), 0, K - 2, K - 1])
    rows = a[:, torch.from_numpy(ids.astype(np.int64)).cuda()].T.contiguous().cpu().numpy()
    oi, oa, ot = oracle.select_ids(rows, ids.astype(np.uint32), seed=9, step=5, threads=8)
    assert np.array_equal(idx.cpu().numpy()[ids], oi)
    assert np.array_equal(tr.cpu().numpy().view(np.uint32)[ids], ot)
    assert np.array_equal(a0.cpu().numpy()[ids].view(np.uint32), oa.view(np.uint32))
    del a
    torch.cuda.empty_cache()


def test_index_only_bench_configuration(gpu):
    """The timed configuration writes indices only (no alpha_0, no trial
    counts): R=4096 x M=1029 SoA, checked against the oracle's indices."""
    M, K = 1029, 4096
    buf = workloads.lognormal_soa(M=M, K=K, seed=2, buffers=2)
    dev = torch.from_numpy(buf).cuda()
    idx = torch.empty(K, dtype=torch.int32, device="cuda")
    for b, step in ((0, 7), (1, 500)):
        arsel.select(dev[b], M, K, K, SOA, seed=1, step=step, index=idx)
        torch.cuda.synchronize()
        oi, _, _ = oracle.select_uniform(buf[b], M, K, K, SOA, seed=1, step=step, threads=8)
        assert np.array_equal(idx.cpu().numpy(), oi), (b, step)
