"""GPU parity of the full SSA run (direct method: AR selection, time step,
stoichiometry, dependency-graph propensity updates) against the CPU oracle:
states, selections and times bit for bit (the time step's ln and alpha_0 are
fixed to one arithmetic on both sides)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_1404_0027_amd import learned, workloads

pytestmark = pytest.mark.gpu


def _deps_expected(net):
    r0, r1, p0, p1 = (np.asarray(v) for v in (net.r0, net.r1, net.p0, net.p1))
    out = []
    for j in range(net.M):
        changed = {int(v) for v in (r0[j], r1[j], p0[j], p1[j]) if v >= 0}
        out.append([i for i in range(net.M) if int(r0[i]) in changed or (r1[i] >= 0 and int(r1[i]) in changed)])
    return out


def test_dependency_graph(gpu):
    net = workloads.mass_action_network()
    dn = learned.DeviceNetwork(net)
    d, n = (v.cpu().numpy() for v in dn.deps())
    want = _deps_expected(net)
    for j in range(net.M):
        if len(want[j]) > 64:
            assert n[j] == -1
        else:
            assert n[j] == len(want[j]) and list(d[j, :n[j]]) == want[j], j


def _run_both(net, X0, *, seed, step0, steps, want_times=True, period=1, t_max=4096):
    dn = learned.DeviceNetwork(net)
    X = torch.from_numpy(X0).cuda()
    t = torch.zeros(X0.shape[0], dtype=torch.float64, device="cuda")
    fired, times = dn.run(X, t, seed=seed, step0=step0, steps=steps, want_fired=True,
                          want_times=want_times, period=period, t_max=t_max)
    xo, to, fo, tmo = oracle.ssa_run(net, X0, seed=seed, step0=step0, steps=steps,
                                     want_times=want_times, threads=8, period=period, t_max=t_max)
    assert np.array_equal(fired.cpu().numpy(), fo)
    assert np.array_equal(X.cpu().numpy(), xo)
    np.testing.assert_array_equal(t.cpu().numpy(), to)
    if want_times:
        np.testing.assert_array_equal(times.cpu().numpy(), tmo)
    return X, t


@pytest.mark.parametrize("period", [1, 7, 64])
@pytest.mark.parametrize("N,M,R,steps", [(64, 100, 40, 300), (641, 1029, 64, 200), (64, 100, 37, 150),
                                         (64, 100, 1, 150), (641, 1029, 9, 100)])
def test_run_matches_oracle(gpu, N, M, R, steps, period):
    """Two realizations share a wavefront: odd R leaves the last one alone."""
    net = workloads.mass_action_network(N=N, M=M, seed=4)
    X0 = workloads.poisson_counts(N=N, R=R, seed=5)
    _run_both(net, X0, seed=3, step0=11, steps=steps, period=period)


@pytest.mark.parametrize("period", [1, 7, 64])
def test_run_times_with_rates_over_120_binades(gpu, period):
    """Rates log-uniform over 2^-110 .. 2^10: the fixed-point alpha_0 drops
    the parts below its scale's resolution, so the times depend on the scale
    exponent's history (set at exact steps, dropped when a propensity reaches
    2^E, taken again at the next step that fires), which both sides follow."""
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    rng = np.random.default_rng(21)
    net = dataclasses.replace(net, rate=(2.0 ** rng.uniform(-110, 10, 100)).astype(np.float32))
    X0 = workloads.poisson_counts(N=64, R=37, seed=5)
    _run_both(net, X0, seed=8, step0=3, steps=400, period=period)
    Q = _shaped_q(net, X0)
    _run_both_q(net, X0, Q, seed=8, step0=3, steps=200, period=period)


@pytest.mark.parametrize("period", [1, 7, 64])
def test_run_times_after_a_propensity_collapse(gpu, period):
    """A 2^60 propensity fires first and vanishes; between exact steps the
    scale stays at 2^61 and alpha_0 keeps about 17 bits of the remaining
    propensities near 2^-47, identically on both sides."""
    i32 = lambda v: np.array(v, np.int32)
    net = workloads.Network(N=3, r0=i32([0, 1, 2]), r1=i32([-1, -1, -1]), p0=i32([2, 2, 1]),
                            p1=i32([-1, -1, -1]),
                            rate=np.array([2.0 ** 60, 1.2345e-15, 1.3e-15], np.float32))
    X0 = np.tile(np.array([[1, 5, 0]], np.int32), (37, 1))
    _run_both(net, X0, seed=5, step0=1, steps=100, period=period)
    _run_both_q(net, X0, np.full((37, 3), 7, np.uint32), seed=5, step0=1, steps=100, period=period)


@pytest.mark.parametrize("kind", ["huge", "subnormal"])
@pytest.mark.parametrize("period", [1, 7, 64])
def test_run_times_at_the_ends_of_the_float_range(gpu, period, kind):
    """alpha_max near FLT_MAX (scale exponent 127 and 128, negative shifts)
    and all-subnormal propensities (shifts above 250)."""
    from test_oracle_time_step import rated_network
    net = rated_network(kind)
    X0 = workloads.poisson_counts(N=24, R=37, seed=2)
    _run_both(net, X0, seed=3, step0=0, steps=120, period=period)
    Q = _shaped_q(net, X0)
    _run_both_q(net, X0, Q, seed=3, step0=0, steps=120, period=period)


@pytest.mark.parametrize("period", [1, 16])
@pytest.mark.parametrize("steps", [1, 31, 32, 33, 63, 64, 65, 128, 129])
def test_run_time_batches_at_their_boundaries(gpu, period, steps):
    """The time step is taken in batches of 64 steps (32 per half with two
    realizations per wavefront): runs ending just before, at and after a
    batch boundary record the oracle's times."""
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    X0 = workloads.poisson_counts(N=64, R=37, seed=5)
    _run_both(net, X0, seed=12, step0=7, steps=steps, period=period)


def test_run_absorbs_and_overflowing_dependency_lists(gpu):
    # pure decay: absorbed after n firings (time stays, -1 recorded)
    dec = workloads.Network(N=2, r0=np.array([0], np.int32), r1=np.array([-1], np.int32),
                            p0=np.array([1], np.int32), p1=np.array([-1], np.int32),
                            rate=np.array([0.5], np.float32))
    X0 = np.tile(np.array([[5, 0]], np.int32), (100, 1))
    _run_both(dec, X0, seed=1, step0=0, steps=9)
    _run_both(dec, X0, seed=1, step0=0, steps=9, period=1000)
    # every reaction consumes species 0: dependency lists overflow (full recompute)
    rng = np.random.default_rng(3)
    M = 150
    hub = workloads.Network(N=4, r0=np.zeros(M, np.int32),
                            r1=rng.integers(-1, 4, M).astype(np.int32),
                            p0=rng.integers(0, 4, M).astype(np.int32),
                            p1=np.full(M, -1, np.int32),
                            rate=rng.lognormal(0, 1, M).astype(np.float32))
    hub.p1[hub.r1 >= 0] = rng.integers(0, 4, int((hub.r1 >= 0).sum()))
    _, n = learned.DeviceNetwork(hub).deps()
    assert (n.cpu().numpy() == -1).any()
    X0 = rng.integers(20, 60, size=(30, 4)).astype(np.int32)
    _run_both(hub, X0, seed=2, step0=5, steps=200)
    _run_both(hub, X0, seed=2, step0=5, steps=200, period=32)


def test_run_resumes_in_segments(gpu):
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    X0 = workloads.poisson_counts(N=64, R=32, seed=6)
    dn = learned.DeviceNetwork(net)
    Xa = torch.from_numpy(X0).cuda()
    ta = torch.zeros(32, dtype=torch.float64, device="cuda")
    dn.run(Xa, ta, seed=4, step0=0, steps=240)
    Xb = torch.from_numpy(X0).cuda()
    tb = torch.zeros(32, dtype=torch.float64, device="cuda")
    dn.run(Xb, tb, seed=4, step0=0, steps=100)
    dn.run(Xb, tb, seed=4, step0=100, steps=140)
    assert torch.equal(Xa, Xb)
    assert torch.equal(ta, tb)


def test_run_resumes_at_period_boundaries(gpu):
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    X0 = workloads.poisson_counts(N=64, R=32, seed=6)
    dn = learned.DeviceNetwork(net)
    Xa = torch.from_numpy(X0).cuda()
    ta = torch.zeros(32, dtype=torch.float64, device="cuda")
    fa, _ = dn.run(Xa, ta, seed=4, step0=0, steps=256, period=64, want_fired=True)
    Xb = torch.from_numpy(X0).cuda()
    tb = torch.zeros(32, dtype=torch.float64, device="cuda")
    f1, _ = dn.run(Xb, tb, seed=4, step0=0, steps=128, period=64, want_fired=True)
    f2, _ = dn.run(Xb, tb, seed=4, step0=128, steps=128, period=64, want_fired=True)
    assert torch.equal(Xa, Xb) and torch.equal(fa, torch.cat([f1, f2]))
    assert torch.equal(ta, tb)


def test_run_graph_capture_replays_match_eager(gpu):
    """Full runs captured in one HIP graph (uniform with maintained envelopes,
    uniform exact every step, proposal), replayed four times from reset states
    with eager runs between the replays: every replay equals the oracle
    (states, times, selections)."""
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    X0 = workloads.poisson_counts(N=64, R=37, seed=5)
    Q = _shaped_q(net, X0)
    dn = learned.DeviceNetwork(net)
    cases = [dict(period=64), dict(period=1), dict(period=16, Q=Q, qfloor=40)]
    refs = []
    for cfg in cases:
        xo, to, fo, tmo = oracle.ssa_run(net, X0, seed=9, step0=5, steps=150, want_times=True,
                                         threads=8, **cfg)
        refs.append((xo, to, fo, tmo))
    Qd = torch.from_numpy(Q.view(np.int32)).cuda()
    X0d = torch.from_numpy(X0).cuda()
    Xs = [X0d.clone() for _ in cases]
    ts = [torch.zeros(37, dtype=torch.float64, device="cuda") for _ in cases]

    def run_all():
        out = []
        for X, t, cfg in zip(Xs, ts, cases):
            kw = dict(period=cfg["period"])
            if "Q" in cfg:
                kw.update(Q=Qd, qfloor=cfg["qfloor"])
            out.append(dn.run(X, t, seed=9, step0=5, steps=150, want_fired=True,
                              want_times=True, **kw))
        return out

    run_all()                       # sizes the context's buffers before the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap, capture_error_mode="relaxed"):
            outs = run_all()
    torch.cuda.synchronize()
    for rep in range(4):
        for X, t in zip(Xs, ts):
            X.copy_(X0d)
            t.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, ((fired, times), (xo, to, fo, tmo)) in enumerate(zip(outs, refs)):
            assert np.array_equal(Xs[i].cpu().numpy(), xo), ("states", i, rep)
            np.testing.assert_array_equal(ts[i].cpu().numpy(), to)
            assert np.array_equal(fired.cpu().numpy(), fo), ("selections", i, rep)
            np.testing.assert_array_equal(times.cpu().numpy(), tmo)
        # eager work between replays, on other buffers and another network
        other = workloads.mass_action_network(N=32, M=70, seed=rep)
        Xe = torch.from_numpy(workloads.poisson_counts(N=32, R=9, seed=rep)).cuda()
        learned.DeviceNetwork(other).run(Xe, torch.zeros(9, dtype=torch.float64, device="cuda"),
                                         seed=1, step0=0, steps=40, period=8)
        torch.cuda.synchronize()


def _sample_ids(R, n, seed):
    """n realization ids: half even, half odd (the two halves of a wavefront in
    the two-realizations-per-wavefront kernel), plus the first and the last."""
    rng = np.random.default_rng(seed)
    ev = 2 * rng.choice(R // 2, n // 2, replace=False)
    od = 2 * rng.choice(R // 2, n // 2, replace=False) + 1
    return np.unique(np.r_[ev, od, 0, R - 1]).astype(np.uint32)


@pytest.mark.parametrize("period", [1, 64])
def test_run_full_size_sampled(gpu, period):
    """R = 16384 realizations x 10^4 steps of the N=641, M=1029 network in one
    launch; 1024 realizations (512 even and 512 odd ids, plus the first and
    the last) replayed by the oracle (instance ids kept)."""
    net = workloads.mass_action_network()
    R, steps = 16384, 10000
    X0 = workloads.poisson_counts(N=net.N, R=R, seed=5)
    dn = learned.DeviceNetwork(net)
    X = torch.from_numpy(X0).cuda()
    t = torch.zeros(R, dtype=torch.float64, device="cuda")
    dn.run(X, t, seed=7, step0=0, steps=steps, period=period)
    torch.cuda.synchronize()
    ids = _sample_ids(R, 1024, seed=period)
    xo, to, _, _ = oracle.ssa_run(net, X0[ids], seed=7, step0=0, steps=steps, ids=ids, threads=16,
                                  period=period)
    assert np.array_equal(X.cpu().numpy()[ids], xo)
    np.testing.assert_array_equal(t.cpu().numpy()[ids], to)
    assert np.array_equal(X.cpu().numpy().sum(axis=1), X0.sum(axis=1))


# ---- the run with an integer proposal (Q' = max(Q, 1), tag-1 stream) ----

def _shaped_q(net, X0):
    """A proposal shaped like the initial propensities (what a trained
    network approximates): alpha quantised to 16 bits of its row maximum,
    zero where the reaction is inactive."""
    a = oracle.propensities(net, X0).astype(np.float64)
    amax = a.max(axis=1, keepdims=True)
    return np.floor(a / np.where(amax > 0, amax, 1.0) * 65535.0).astype(np.uint32)


def _run_both_q(net, X0, Q, *, seed, step0, steps, t_max=4096, ldq=None, want_times=True,
                qfloor=1, period=1):
    R, M = Q.shape
    ldq = ldq or M
    Qp = np.zeros((R, ldq), np.uint32)
    Qp[:, :M] = Q
    Qp[:, M:] = 0xDEADBEEF                      # padding is never read
    dn = learned.DeviceNetwork(net)
    X = torch.from_numpy(X0).cuda()
    t = torch.zeros(R, dtype=torch.float64, device="cuda")
    Qd = torch.from_numpy(Qp.view(np.int32)).cuda()
    fired, times = dn.run(X, t, seed=seed, step0=step0, steps=steps, t_max=t_max, want_fired=True,
                          want_times=want_times, Q=Qd, qfloor=qfloor, period=period)
    xo, to, fo, tmo = oracle.ssa_run(net, X0, seed=seed, step0=step0, steps=steps, t_max=t_max,
                                     want_times=want_times, threads=8, Q=Q, qfloor=qfloor,
                                     period=period)
    assert np.array_equal(fired.cpu().numpy(), fo)
    assert np.array_equal(X.cpu().numpy(), xo)
    np.testing.assert_array_equal(t.cpu().numpy(), to)
    if want_times:
        np.testing.assert_array_equal(times.cpu().numpy(), tmo)
    return fo


@pytest.mark.parametrize("period", [1, 16])
@pytest.mark.parametrize("kind,qfloor", [("random", 1), ("shaped", 1), ("shaped", 80),
                                         ("random", 0xFFFFFFFF // 1000)])
@pytest.mark.parametrize("N,M,R,steps", [(64, 100, 40, 300), (641, 1029, 64, 200)])
def test_run_with_proposal_matches_oracle(gpu, N, M, R, steps, kind, qfloor, period):
    net = workloads.mass_action_network(N=N, M=M, seed=4)
    X0 = workloads.poisson_counts(N=N, R=R, seed=5)
    if kind == "random":
        rng = np.random.default_rng(M)
        Q = rng.integers(0, 1000, size=(R, M)).astype(np.uint32)
        Q[rng.random((R, M)) < 0.2] = 0
    else:
        Q = _shaped_q(net, X0)
    fo = _run_both_q(net, X0, Q, seed=3, step0=11, steps=steps, qfloor=qfloor, period=period)
    # a floor with sum Q' >= 2^32 (the last case at M = 1029) stops every realization
    assert np.all(fo == -4) == (qfloor * M >= 2**32)


@pytest.mark.parametrize("t_max", [0, 1, 3])
def test_run_with_proposal_budgets_and_padding(gpu, t_max):
    """Short trial budgets (fallback inverse transform) and ldq > M."""
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    X0 = workloads.poisson_counts(N=64, R=48, seed=7)
    Q = _shaped_q(net, X0)
    _run_both_q(net, X0, Q, seed=5, step0=2, steps=120, t_max=t_max, ldq=107)
    _run_both_q(net, X0, Q, seed=5, step0=2, steps=120, t_max=t_max, ldq=107, period=50)
    # the uniform run's fallback, with exact and maintained envelopes, odd R
    _run_both(net, X0, seed=5, step0=2, steps=120, period=50, t_max=t_max)
    _run_both(net, X0[:47], seed=6, step0=2, steps=120, period=1, t_max=t_max)


def test_run_with_proposal_overflow_and_absorption(gpu):
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    X0 = workloads.poisson_counts(N=64, R=32, seed=8)
    Q = _shaped_q(net, X0)
    Q[:10] = 0xFFFFFFFF                         # sum Q' >= 2^32: -4, nothing moves
    fo = _run_both_q(net, X0, Q, seed=6, step0=0, steps=50)
    assert np.all(fo[:, :10] == -4) and np.all(fo[:, 10:] >= 0)
    dec = workloads.Network(N=2, r0=np.array([0], np.int32), r1=np.array([-1], np.int32),
                            p0=np.array([1], np.int32), p1=np.array([-1], np.int32),
                            rate=np.array([0.5], np.float32))
    X0 = np.tile(np.array([[5, 0]], np.int32), (64, 1))
    fo = _run_both_q(dec, X0, np.zeros((64, 1), np.uint32), seed=1, step0=0, steps=9)
    assert np.all(fo[:5] == 0) and np.all(fo[5:] == -1)


def test_run_with_proposal_argument_errors(gpu):
    import ctypes

    from paper_1404_0027_amd import arsel
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    dn = learned.DeviceNetwork(net)
    d, n = dn.deps()
    X = torch.from_numpy(workloads.poisson_counts(N=64, R=4, seed=1)).cuda()
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    Q = torch.ones(4, 100, dtype=torch.int32, device="cuda")
    call = lambda q, ldq: arsel.lib().arsel_ssa_run_proposal(
        arsel.context(0), ctypes.byref(dn.c), d.data_ptr(), n.data_ptr(), q, ldq, 1, X.data_ptr(), 4,
        1, 0, 5, 4096, 1, t.data_ptr(), None, None, torch.cuda.current_stream().cuda_stream)
    assert call(None, 100) == -1                  # Q NULL
    assert call(Q.data_ptr(), 99) == -4           # ldq < M
    assert call(Q.data_ptr(), 100) == 0
    with pytest.raises(arsel.ArselError):
        dn.run(X, t, seed=1, step0=0, steps=1, Q=Q[:, :99].contiguous())


def test_run_with_proposal_full_size_sampled(gpu):
    """R = 16384 x 10^4 steps with the proposal shaped on the initial states;
    258 realizations (even and odd ids, the first and the last) replayed by
    the oracle (instance ids kept)."""
    net = workloads.mass_action_network()
    R, steps = 16384, 10000
    X0 = workloads.poisson_counts(N=net.N, R=R, seed=5)
    ids = _sample_ids(R, 256, seed=9)
    Q = np.zeros((R, net.M), np.uint32)
    Q[ids] = _shaped_q(net, X0[ids])
    Q[np.setdiff1d(np.arange(R), ids)] = 3
    dn = learned.DeviceNetwork(net)
    X = torch.from_numpy(X0).cuda()
    t = torch.zeros(R, dtype=torch.float64, device="cuda")
    dn.run(X, t, seed=7, step0=0, steps=steps, Q=torch.from_numpy(Q.view(np.int32)).cuda(),
           qfloor=60, period=64)
    torch.cuda.synchronize()
    xo, to, _, _ = oracle.ssa_run(net, X0[ids], seed=7, step0=0, steps=steps, ids=ids, threads=16,
                                  Q=Q[ids], qfloor=60, period=64)
    assert np.array_equal(X.cpu().numpy()[ids], xo)
    np.testing.assert_array_equal(t.cpu().numpy()[ids], to)
    assert np.array_equal(X.cpu().numpy().sum(axis=1), X0.sum(axis=1))


@pytest.mark.parametrize("period", [1, 32])
def test_run_with_the_networks_proposal(gpu, period):
    """The learned pipeline end to end: the MLP's quantised proposal for the
    current states (untrained weights, seed 3) drives the run; the oracle
    replays it on the GPU's Q, so selections, states and times still match."""
    net = workloads.mass_action_network()
    X0 = workloads.poisson_counts(N=net.N, R=24, seed=8)
    X0[:, :64] = 0      # some reactions start inactive and may turn active during the run
    dn = learned.DeviceNetwork(net)
    lp = learned.LearnedProposal(net.N, net.M, seed=3)
    X = torch.from_numpy(X0).cuda()
    Q, _ = lp.forward(X, dn.propensities(X))
    Qh = Q.cpu().numpy().view(np.uint32)
    assert (Qh > 0).any() and (Qh == 0).any()      # zeros where a reaction is inactive
    qfloor = (1 << (31 - (net.M - 1).bit_length())) // (8 * net.M)
    _run_both_q(net, X0, Qh, seed=4, step0=3, steps=150, qfloor=qfloor, period=period)


@pytest.mark.parametrize("period", [1, 64])
def test_run_invalid_propensities(gpu, period):
    """A propensity that turns negative during the run (kept by the
    maintained counts between exact steps) and a NaN rate: -2, as the oracle."""
    i32 = lambda v: np.array(v, np.int32)
    X0 = np.tile(np.array([[5, 0, 0]], np.int32), (9, 1))
    for rate1 in (-1.0, np.nan):
        net = workloads.Network(N=3, r0=i32([0, 1, 2]), r1=i32([-1, -1, -1]), p0=i32([1, 2, 0]),
                                p1=i32([-1, -1, -1]), rate=np.array([1.0, rate1, 1.0], np.float32))
        _run_both(net, X0, seed=2, step0=0, steps=6, period=period)
        Q = np.full((9, 3), 5, np.uint32)
        _run_both_q(net, X0, Q, seed=2, step0=0, steps=6, period=period)


def test_run_argument_errors_and_no_ops(gpu):
    import ctypes

    from paper_1404_0027_amd import arsel
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    dn = learned.DeviceNetwork(net)
    d, n = dn.deps()
    X = torch.from_numpy(workloads.poisson_counts(N=64, R=4, seed=1)).cuda()
    X_before = X.clone()
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    run = lambda dp, xp, R, steps, tp: arsel.lib().arsel_ssa_run(
        arsel.context(0), ctypes.byref(dn.c), dp, n.data_ptr(), xp, R, 1, 0, steps, 4096, 64, tp,
        None, None, st)
    assert run(d.data_ptr(), X.data_ptr(), 0, 10, t.data_ptr()) == 0        # R = 0: nothing
    assert run(d.data_ptr(), X.data_ptr(), 4, 0, t.data_ptr()) == 0         # steps = 0: nothing
    assert run(d.data_ptr(), X.data_ptr(), -1, 10, t.data_ptr()) == -2      # ARSEL_ERR_SIZE
    assert run(d.data_ptr(), X.data_ptr(), 4, -1, t.data_ptr()) == -2
    assert run(None, X.data_ptr(), 4, 10, t.data_ptr()) == -1               # ARSEL_ERR_NULL
    assert run(d.data_ptr(), None, 4, 10, t.data_ptr()) == -1
    assert run(d.data_ptr(), X.data_ptr(), 4, 10, None) == -1
    torch.cuda.synchronize()
    assert torch.equal(X, X_before) and torch.count_nonzero(t) == 0
    bad = arsel.Network(net.N, net.M, None, None, None, None, None)
    assert arsel.lib().arsel_ssa_run(arsel.context(0), ctypes.byref(bad), d.data_ptr(),
                                     n.data_ptr(), X.data_ptr(), 4, 1, 0, 10, 4096, 64,
                                     t.data_ptr(), None, None, st) == -1
