"""GPU parity of arsel_select_ragged (uneven batches) against the CPU oracle,
bit for bit, under several schedules."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_0027_amd import arsel, workloads
from tests.parity import assert_same

pytestmark = pytest.mark.gpu


def _ragged_both(alpha, offsets, *, seed, step, t_max=4096, host=True, ids=None):
    a = torch.from_numpy(np.ascontiguousarray(alpha, np.float32)).cuda()
    off = torch.from_numpy(np.ascontiguousarray(offsets, np.int64)).cuda()
    idx, a0, tr = arsel.select_ragged(a, off, seed=seed, step=step, t_max=t_max,
                                      host_offsets=offsets if host else None,
                                      want_alpha0=True, want_trials=True)
    torch.cuda.synchronize()
    g = (idx.cpu().numpy(), a0.cpu().numpy(), tr.cpu().numpy().view(np.uint32))
    if ids is not None:
        g = tuple(x[ids] for x in g)
    o = oracle.select_ragged(alpha, offsets, seed=seed, step=step, t_max=t_max, ids=ids,
                             threads=8)
    return g, o


def _schedules():
    return [(1024, 8, 8192, 2), (256, 4, 4096, 4), (4096, 8, 16384, 1), (64, 8, 0, 2),
            (2048, 4, 2048, 1)]


@pytest.fixture
def restore_schedule(gpu):
    s0 = arsel.get_schedule()
    yield
    arsel.set_schedule(s0)


def test_ragged_mix_small(gpu):
    rb = workloads.ragged_mix(K=400, seed=3, log2_lo=0, log2_hi=14)
    for host in (True, False):
        g, o = _ragged_both(rb.alpha, rb.offsets, seed=1, step=3, host=host)
        assert_same(g, o, f"ragged host={host}")


@pytest.mark.parametrize("sched", _schedules())
def test_ragged_schedules_do_not_change_results(gpu, restore_schedule, sched):
    rb = workloads.ragged_mix(K=300, seed=31, log2_lo=0, log2_hi=15)
    s = arsel.Schedule(*sched)
    arsel.set_schedule(s)
    g, o = _ragged_both(rb.alpha, rb.offsets, seed=9, step=11)
    assert_same(g, o, f"schedule {sched}")


@pytest.mark.parametrize("t_max", [0, 1, 130, 1024])
def test_ragged_fallbacks(gpu, t_max):
    """Small budgets force the fixed-point fallback in both the wavefront and
    the workgroup paths (staged and gathered from global memory)."""
    rb = workloads.ragged_mix(K=120, seed=5, log2_lo=4, log2_hi=16)
    g, o = _ragged_both(rb.alpha, rb.offsets, seed=2, step=t_max, t_max=t_max)
    assert_same(g, o, f"t_max {t_max}")
    if t_max == 0:
        assert np.all((g[2] == 1) | (g[0] < 0))            # every selection fell back
    if t_max == 1:
        assert np.all((g[2] <= 2) | (g[0] < 0)) and np.any(g[2] == 2)


@pytest.mark.parametrize("sched", [(64, 8, 0, 2), (256, 4, 2048, 1), (1024, 16, 8192, 1)])
def test_ragged_hard_chunks_and_fallbacks(gpu, restore_schedule, sched):
    """Heavy-tailed rows (lognormal, sigma 3) are hard: they are cut into chunks
    of the schedule's piece (2048 floats: up to 32 chunks per row on the
    device-built path, longer rows then take chunks of several pieces), each
    chunk tests every trial whose candidate it holds, and tiny budgets send
    most of them to the fallback, located from the chunk sums."""
    arsel.set_schedule(arsel.Schedule(*sched))
    rng = np.random.default_rng(8)
    sizes = np.round(2 ** rng.uniform(10, 17.5, 60)).astype(np.int64)
    offsets = np.zeros(61, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    alpha = rng.lognormal(0.0, 3.0, int(offsets[-1])).astype(np.float32)
    for host in (True, False):
        for t_max in (0, 3, 4096):
            g, o = _ragged_both(alpha, offsets, seed=6, step=t_max, t_max=t_max, host=host)
            assert_same(g, o, f"schedule {sched} t_max {t_max} host={host}")
    if t_max == 4096:
        assert np.any(g[2] == 4097)          # some rows still fell back


def test_ragged_huge_instance(gpu):
    """One instance of 2^24 + 7 reactions between two small ones: a hard row of
    about a thousand chunks with host lists, and of 32 chunks of several LDS
    pieces each with device-built lists; t_max 4096 and 0 (the fallback is
    located from the chunk sums and searched in one chunk)."""
    rng = np.random.default_rng(22)
    sizes = np.array([5, (1 << 24) + 7, 100], np.int64)
    offsets = np.zeros(4, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    alpha = rng.lognormal(0, 2, int(offsets[-1])).astype(np.float32)
    for host in (True, False):
        for t_max in (4096, 0):
            g, o = _ragged_both(alpha, offsets, seed=3, step=t_max, t_max=t_max, host=host)
            assert_same(g, o, f"huge instance host={host} t_max={t_max}")
    assert g[0][1] >= 0


def test_ragged_edge_instances(gpu):
    rng = np.random.default_rng(7)
    rows = [np.zeros(0), np.zeros(5), np.array([2.0]), rng.random(3000),
            np.r_[rng.random(100), np.nan], np.r_[rng.random(20000), -1.0],
            np.zeros(20000), np.full(70, 3e-44), rng.lognormal(0, 3, 40000),
            np.r_[np.full(10, -0.0), 1.0], np.zeros(0), rng.random(64),
            rng.random(5000) * 1e-40,                      # large, subnormal maximum
            np.r_[rng.lognormal(0, 4, 30000) * 1e-45]]     # large, heavy-tailed subnormals
    sizes = np.array([len(r) for r in rows], np.int64)
    offsets = np.zeros(len(rows) + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    alpha = np.concatenate(rows).astype(np.float32)
    for host in (True, False):
        for t_max in (4096, 0):
            g, o = _ragged_both(alpha, offsets, seed=4, step=1, t_max=t_max, host=host)
            assert_same(g, o, f"edge host={host} t_max={t_max}")
    assert g[0][0] == -1 and g[0][1] == -1 and g[0][2] == 0 and g[0][4] == -2 and g[0][5] == -2
    assert g[0][6] == -1 and g[0][10] == -1 and g[0][9] == 10


def test_ragged_full_size(gpu):
    """10^4 instances, M log-uniform in [64, 65536] (about 9.4e7 propensities):
    the whole batch in one launch, every instance checked against the oracle
    (indices, alpha_0 and trial counts), with and without host sizes."""
    rb = workloads.ragged_mix(K=10000, seed=3)
    for host in (True, False):
        g, o = _ragged_both(rb.alpha, rb.offsets, seed=1, step=0, host=host)
        assert_same(g, o, f"ragged full size host={host}")


def test_ragged_matches_dense(gpu):
    """A ragged batch of equal sizes equals the dense AoS call (same instance ids)."""
    rng = np.random.default_rng(12)
    K, M = 64, 777
    a = rng.exponential(1.0, size=(K, M)).astype(np.float32)
    offsets = np.arange(K + 1, dtype=np.int64) * M
    t = torch.from_numpy(a).cuda()
    d = arsel.select(t, M, K, M, arsel.AOS, seed=3, step=5, want_alpha0=True, want_trials=True)
    r = arsel.select_ragged(t.view(-1), torch.from_numpy(offsets).cuda(), seed=3, step=5,
                            host_offsets=offsets, want_alpha0=True, want_trials=True)
    for x, y in zip(d, r):
        assert torch.equal(x, y)


def test_ragged_argument_errors(gpu):
    a = torch.ones(10, device="cuda")
    with pytest.raises(arsel.ArselError):
        arsel.select_ragged(a, torch.tensor([0, 5, 20], dtype=torch.int64, device="cuda"),
                            seed=1, host_offsets=np.array([0, 5, 20]))   # beyond alpha
    with pytest.raises(arsel.ArselError):
        arsel.select_ragged(a, torch.tensor([0, 5, 3], dtype=torch.int64, device="cuda"),
                            seed=1, host_offsets=np.array([0, 5, 3]))    # decreasing
    bad = arsel.Schedule(1 << 20, 16, 0, 1)                               # LDS too large
    with pytest.raises(arsel.ArselError):
        arsel.set_schedule(bad)


def test_autotuner_picks_a_valid_schedule_and_results_hold(gpu, restore_schedule, tmp_path,
                                                            monkeypatch):
    from paper_1404_0027_amd import autotune

    monkeypatch.setattr(autotune, "CACHE_PATH", str(tmp_path / "cache.json"))
    rb = workloads.ragged_mix(K=500, seed=8, log2_lo=4, log2_hi=16)
    a = torch.from_numpy(rb.alpha).cuda()
    off = torch.from_numpy(rb.offsets).cuda()
    cands = [(256, 4, 0, 1), (1024, 8, 8192, 2), (2048, 8, 16384, 2)]
    res = autotune.tune_ragged(a, off, rb.offsets, candidates=cands, reps=2)
    assert res.schedule in cands and len(res.table) == len(cands)
    assert tuple(arsel.get_schedule().__getattribute__(f) for f in
                 ("wave_max_m", "block_waves", "lds_max_m", "blocks_per_cu")) == res.schedule
    g, o = _ragged_both(rb.alpha, rb.offsets, seed=6, step=2)
    assert_same(g, o, "tuned schedule")
    # cached: the second call does not search
    res2 = autotune.tune_ragged(a, off, rb.offsets, candidates=cands, reps=2)
    assert res2.schedule == res.schedule and res2.table == []


def test_ragged_index_only_bench_configuration(gpu, restore_schedule):
    """The timed configuration (10^4 instances, host sizes, indices only, the
    autotuned schedule) against the oracle on every instance, two steps (the
    second call reuses the device work lists)."""
    from paper_1404_0027_amd import autotune

    rb = workloads.ragged_mix(K=10000, seed=3)
    a = torch.from_numpy(rb.alpha).cuda()
    off = torch.from_numpy(rb.offsets).cuda()
    autotune.tune_ragged(a, off, rb.offsets, reps=2, use_cache=False)
    idx = torch.empty(rb.K, dtype=torch.int32, device="cuda")
    for step in (2, 3):
        arsel.select_ragged(a, off, seed=1, step=step, host_offsets=rb.offsets, index=idx)
        torch.cuda.synchronize()
        oi, _, _ = oracle.select_ragged(rb.alpha, rb.offsets, seed=1, step=step, threads=8)
        assert np.array_equal(idx.cpu().numpy(), oi), step


def _sized_batch(seed, K=500):
    r = np.random.default_rng(seed)
    sizes = np.round(2 ** r.uniform(0, 14, K)).astype(np.int64)
    offsets = np.zeros(K + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    alpha = r.exponential(1.0, int(offsets[-1])).astype(np.float32)
    return alpha, offsets


def test_ragged_work_lists_reused_only_for_equal_sizes(gpu):
    """Calls with the same K alternate between sizes, values and the
    device-built lists: reused lists never serve other sizes."""
    A, B = _sized_batch(1), _sized_batch(2)
    A2 = (np.random.default_rng(3).random(A[0].shape[0]).astype(np.float32), A[1])
    seq = [(A, True), (A, True), (B, True), (A2, True), (A, False), (A, True), (B, False), (B, True)]
    for n, ((alpha, offsets), host) in enumerate(seq):
        g, o = _ragged_both(alpha, offsets, seed=3, step=n, host=host)
        assert_same(g, o, f"call {n} host={host}")


def test_ragged_counters_cleared_between_calls(gpu):
    """Thirty calls in a row on one stream, outputs pre-filled with a sentinel:
    every call covers every instance (each call's scan kernel zeroes the
    counters its split kernel fills)."""
    alpha, offsets = _sized_batch(4)
    a = torch.from_numpy(alpha).cuda()
    off = torch.from_numpy(offsets).cuda()
    K = offsets.shape[0] - 1
    oi, _, _ = oracle.select_ragged(alpha, offsets, seed=5, step=9, threads=8)
    outs = torch.full((30, K), -7, dtype=torch.int32, device="cuda")
    for n in range(30):
        arsel.select_ragged(a, off, seed=5, step=9, host_offsets=offsets if n % 3 else None,
                            index=outs[n])
    torch.cuda.synchronize()
    for n in range(30):
        assert np.array_equal(outs[n].cpu().numpy(), oi), n


def test_ragged_graph_capture_replays_match_eager(gpu):
    """Captured calls (host sizes whose lists were built eagerly, host sizes
    never seen before, device-built lists) replayed several times with eager
    calls between the replays that rebuild the host lists for other sizes and
    outgrow the device list buffer: every replay equals the oracle (under
    capture the lists are built inside the graph; outgrown buffers are kept
    while the context lives)."""
    A, B = _sized_batch(11), _sized_batch(12)
    C = _sized_batch(13, K=3000)
    a = torch.from_numpy(A[0]).cuda()
    off = torch.from_numpy(A[1]).cuda()
    b = torch.from_numpy(B[0]).cuda()
    offb = torch.from_numpy(B[1]).cuda()
    c = torch.from_numpy(C[0]).cuda()
    offc = torch.from_numpy(C[1]).cuda()
    K, KB = A[1].shape[0] - 1, B[1].shape[0] - 1
    ref, _, _ = oracle.select_ragged(A[0], A[1], seed=8, step=4, threads=8)
    refb, _, _ = oracle.select_ragged(B[0], B[1], seed=6, step=2, threads=8)
    arsel.select_ragged(a, off, seed=8, step=4, host_offsets=A[1])       # eager: lists built
    torch.cuda.synchronize()
    out_h = torch.full((K,), -7, dtype=torch.int32, device="cuda")
    out_d = torch.full((K,), -7, dtype=torch.int32, device="cuda")
    out_b = torch.full((KB,), -7, dtype=torch.int32, device="cuda")
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap, capture_error_mode="relaxed"):
            arsel.select_ragged(a, off, seed=8, step=4, host_offsets=A[1], index=out_h)
            arsel.select_ragged(a, off, seed=8, step=4, index=out_d)
            arsel.select_ragged(b, offb, seed=6, step=2, host_offsets=B[1], index=out_b)
    torch.cuda.synchronize()
    for rep in range(4):
        for o in (out_h, out_d, out_b):
            o.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out_h.cpu().numpy(), ref), ("host sizes, built before", rep)
        assert np.array_equal(out_d.cpu().numpy(), ref), ("device lists", rep)
        assert np.array_equal(out_b.cpu().numpy(), refb), ("host sizes, not built before", rep)
        # eager work between replays: host lists for other sizes, then a larger
        # batch with device-built lists (the list buffers grow)
        arsel.select_ragged(b, offb, seed=1, step=rep, host_offsets=B[1])
        oc, _, _ = arsel.select_ragged(c, offc, seed=1, step=rep)
        torch.cuda.synchronize()
    # the context still serves eager calls after the replays
    g_, o_ = _ragged_both(B[0], B[1], seed=2, step=3)
    assert_same(g_, o_, "after the replays")
    g_, o_ = _ragged_both(A[0], A[1], seed=2, step=5, host=False)
    assert_same(g_, o_, "device lists after the replays")


@pytest.mark.parametrize("sched", [(1024, 8, 8192, 2), (256, 4, 0, 4), (2048, 16, 16384, 1)])
def test_ragged_sub_batch_and_chunked_rows(gpu, restore_schedule, sched):
    """A batch whose offsets start inside alpha (offsets[0] > 0, odd sizes, so
    rows and chunks start at every alignment) with rows of up to 2^17
    elements, cut into several chunks by every schedule: host and device
    lists against the oracle."""
    r = np.random.default_rng(41)
    K = 160
    sizes = np.round(2 ** r.uniform(0, 17, K)).astype(np.int64)
    sizes[[3, 50]] = [131071, 70001]                 # many chunks, odd lengths
    offsets = np.zeros(K + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    offsets += 37                                      # the batch starts inside alpha
    fam = r.integers(0, 3, K)
    alpha = np.empty(int(offsets[-1]) + 5, np.float32)
    alpha[:37] = np.nan                                # never read
    for k in range(K):
        m = int(sizes[k])
        v = [1.0 - r.random(m), r.exponential(1.0, m), r.lognormal(0.0, 3.0, m)][fam[k]]
        alpha[offsets[k]:offsets[k + 1]] = v
    alpha[-5:] = np.nan
    arsel.set_schedule(arsel.Schedule(*sched))
    for host in (True, False):
        g, o = _ragged_both(alpha, offsets, seed=4, step=2, host=host)
        assert_same(g, o, f"schedule {sched} host={host}")


def test_ragged_device_lists_large_batch(gpu):
    """More than 65536 instances with device-built lists (reset + unordered
    split) and with host sizes: every instance against the oracle."""
    r = np.random.default_rng(21)
    K = 70000
    sizes = np.round(2 ** r.uniform(0, 9, K)).astype(np.int64)
    offsets = np.zeros(K + 1, np.int64)
    np.cumsum(sizes, out=offsets[1:])
    alpha = r.exponential(1.0, int(offsets[-1])).astype(np.float32)
    for host in (False, True, False):
        g, o = _ragged_both(alpha, offsets, seed=3, step=1, host=host)
        assert_same(g, o, f"K={K} host={host}")
