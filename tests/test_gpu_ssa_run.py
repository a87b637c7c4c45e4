"""GPU parity of the full SSA run (direct method: AR selection, time step,
stoichiometry, dependency-graph propensity updates) against the CPU oracle:
states and selections bit for bit, times to rounding."""
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


def _run_both(net, X0, *, seed, step0, steps, want_times=True):
    dn = learned.DeviceNetwork(net)
    X = torch.from_numpy(X0).cuda()
    t = torch.zeros(X0.shape[0], dtype=torch.float64, device="cuda")
    fired, times = dn.run(X, t, seed=seed, step0=step0, steps=steps, want_fired=True,
                          want_times=want_times)
    xo, to, fo, tmo = oracle.ssa_run(net, X0, seed=seed, step0=step0, steps=steps,
                                     want_times=want_times, threads=8)
    assert np.array_equal(fired.cpu().numpy(), fo)
    assert np.array_equal(X.cpu().numpy(), xo)
    np.testing.assert_allclose(t.cpu().numpy(), to, rtol=1e-12, atol=0)
    if want_times:
        np.testing.assert_allclose(times.cpu().numpy(), tmo, rtol=1e-12, atol=0)
    return X, t


@pytest.mark.parametrize("N,M,R,steps", [(64, 100, 40, 300), (641, 1029, 64, 200)])
def test_run_matches_oracle(gpu, N, M, R, steps):
    net = workloads.mass_action_network(N=N, M=M, seed=4)
    X0 = workloads.poisson_counts(N=N, R=R, seed=5)
    _run_both(net, X0, seed=3, step0=11, steps=steps)


def test_run_absorbs_and_overflowing_dependency_lists(gpu):
    # pure decay: absorbed after n firings (time stays, -1 recorded)
    dec = workloads.Network(N=2, r0=np.array([0], np.int32), r1=np.array([-1], np.int32),
                            p0=np.array([1], np.int32), p1=np.array([-1], np.int32),
                            rate=np.array([0.5], np.float32))
    X0 = np.tile(np.array([[5, 0]], np.int32), (100, 1))
    _run_both(dec, X0, seed=1, step0=0, steps=9)
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
    np.testing.assert_allclose(ta.cpu().numpy(), tb.cpu().numpy(), rtol=1e-13)


def test_run_full_size_sampled(gpu):
    """R = 16384 realizations x 10^4 steps of the N=641, M=1029 network in one
    launch; four realizations replayed by the oracle (instance ids kept)."""
    net = workloads.mass_action_network()
    R, steps = 16384, 10000
    X0 = workloads.poisson_counts(N=net.N, R=R, seed=5)
    dn = learned.DeviceNetwork(net)
    X = torch.from_numpy(X0).cuda()
    t = torch.zeros(R, dtype=torch.float64, device="cuda")
    dn.run(X, t, seed=7, step0=0, steps=steps)
    torch.cuda.synchronize()
    ids = np.array([0, 5001, 12345, R - 1], np.uint32)
    xo, to, _, _ = oracle.ssa_run(net, X0[ids], seed=7, step0=0, steps=steps, ids=ids, threads=4)
    assert np.array_equal(X.cpu().numpy()[ids], xo)
    np.testing.assert_allclose(t.cpu().numpy()[ids], to, rtol=1e-9, atol=0)
    assert np.array_equal(X.cpu().numpy().sum(axis=1), X0.sum(axis=1))
