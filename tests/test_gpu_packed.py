"""GPU parity of the broadcast kernels with packed rounds (one vector, K
instances, L lanes per instance) against the CPU oracle, bit for bit, for
every trial width; and the law of the learned proposal in that mode."""
import numpy as np
import pytest
import torch

import oracle
from oracle import laws
from paper_1404_0027_amd import arsel, learned, workloads
from tests.parity import assert_same

pytestmark = pytest.mark.gpu

LANES = [0, 1, 2, 4, 8, 16, 32, 64]


@pytest.fixture
def restore_lanes(gpu):
    yield
    arsel.set_trial_lanes(0)


def _uniform_both(alpha, K, *, seed, step, t_max=4096):
    a = torch.from_numpy(np.ascontiguousarray(alpha, np.float32)).cuda()
    idx, a0, tr = arsel.select(a, alpha.size, K, 0, arsel.AOS, seed=seed, step=step, t_max=t_max,
                               want_alpha0=True, want_trials=True)
    torch.cuda.synchronize()
    g = (idx.cpu().numpy(), a0.cpu().numpy(), tr.cpu().numpy().view(np.uint32))
    o = oracle.select_uniform(alpha, alpha.size, K, 0, oracle.AOS, seed=seed, step=step,
                              t_max=t_max, threads=8)
    return g, o


@pytest.mark.parametrize("lanes", LANES)
def test_packed_uniform_every_width(restore_lanes, lanes):
    arsel.set_trial_lanes(lanes)
    cases = [(workloads.uniform_vector(M=16, seed=1), 1024, 4096),          # config-1 shape
             (workloads.lognormal_soa(M=1029, K=1, seed=2)[:, 0].copy(), 3000, 4096),
             (workloads.lognormal_soa(M=1029, K=1, seed=2)[:, 0].copy(), 777, 5),    # budget hits
             (np.r_[np.zeros(40, np.float32), np.float32(3.0)], 130, 4096)]         # one active
    for alpha, K, t_max in cases:
        g, o = _uniform_both(alpha, K, seed=3, step=lanes + 7, t_max=t_max)
        assert_same(g, o, f"lanes {lanes} M {alpha.size} K {K} t_max {t_max}")


@pytest.mark.parametrize("lanes", [0, 1, 64])
def test_packed_uniform_status_and_fallback(restore_lanes, lanes):
    arsel.set_trial_lanes(lanes)
    for alpha in (np.zeros(33, np.float32),                                   # -1
                  np.array([1.0, np.nan, 2.0], np.float32),                   # -2
                  np.array([1.0, -0.0, 2.0], np.float32),                     # -0.0 is zero
                  np.array([0.5, 1e-30, 2.0, 1e-40], np.float32)):
        for t_max in (0, 1, 4096):
            g, o = _uniform_both(alpha, 300, seed=5, step=t_max, t_max=t_max)
            assert_same(g, o, f"lanes {lanes} alpha {alpha} t_max {t_max}")


def _proposal_both(alpha, Q, K, *, seed, step, t_max=4096):
    a = torch.from_numpy(np.ascontiguousarray(alpha, np.float32)).cuda()
    q = torch.from_numpy(np.ascontiguousarray(Q, np.uint32).view(np.int32)).cuda()
    idx, tr = arsel.select_proposal_broadcast(a, q, K, seed=seed, step=step, t_max=t_max,
                                              want_trials=True)
    torch.cuda.synchronize()
    g = (idx.cpu().numpy(), tr.cpu().numpy().view(np.uint32))
    o = oracle.select_proposal_broadcast(alpha, Q, K, seed=seed, step=step, t_max=t_max,
                                         threads=8)
    return g, o


def _proposal_case(M=1029, seed=0, noise=0.3):
    rng = np.random.default_rng(seed)
    alpha = rng.lognormal(0.0, 2.0, M).astype(np.float32)
    alpha[rng.random(M) < 0.3] = 0.0
    q = np.where(alpha > 0, alpha * np.exp(noise * rng.normal(size=M)), 0.0)
    q = q / q.sum()
    L = laws.ceil_log2(M)
    Q = np.where(alpha > 0, np.maximum(np.floor(q * 2.0 ** (31 - L)), 1), 0).astype(np.uint32)
    return alpha, Q


@pytest.mark.parametrize("lanes", LANES)
def test_packed_proposal_every_width(restore_lanes, lanes):
    arsel.set_trial_lanes(lanes)
    alpha, Q = _proposal_case()
    for K, t_max in ((5000, 4096), (640, 3), (129, 0)):
        g, o = _proposal_both(alpha, Q, K, seed=11, step=lanes, t_max=t_max)
        assert np.array_equal(g[0], o[0]), (lanes, K, t_max)
        assert np.array_equal(g[1], o[1]), (lanes, K, t_max)


def test_packed_proposal_status(restore_lanes):
    alpha, Q = _proposal_case(M=200, seed=4)
    bad = [(alpha.copy(), Q.copy()) for _ in range(4)]
    bad[0][1][np.argmax(alpha)] = 0                      # support not covered: -4
    bad[1][1][:] = 0
    bad[1][1][0] = 0xFFFFFFFF
    bad[1][1][1] = 2                                     # sum Q >= 2^32: -4 (or -1 first)
    bad[2][0][7] = np.inf                                # -2
    bad[3][0][:] = 0                                     # -1
    for lanes in (0, 1, 8):
        arsel.set_trial_lanes(lanes)
        for a, q in bad:
            g, o = _proposal_both(a, q, 100, seed=1, step=2)
            assert np.array_equal(g[0], o[0]) and np.array_equal(g[1], o[1])


def test_packed_proposal_law(restore_lanes):
    """2.56e5 learned-mode selections from one vector follow alpha_j / alpha_0
    (chi-square against the exact law on the 2^-32 grid)."""
    alpha, Q = _proposal_case(M=64, seed=9, noise=0.5)
    a = torch.from_numpy(alpha).cuda()
    q = torch.from_numpy(Q.view(np.int32)).cuda()
    counts = np.zeros(64)
    for step in range(4):
        idx, _ = arsel.select_proposal_broadcast(a, q, 65536, seed=21, step=step)
        counts += np.bincount(idx.cpu().numpy(), minlength=64)
    law, _ = laws.proposal_law(alpha, Q, 4096)
    assert laws.chi_square_p(counts, law) > 0.01


def test_packed_matches_per_instance_kernels(restore_lanes):
    """The broadcast proposal kernel and the one-wavefront kernel on a
    materialised [K, M] copy give the same bits."""
    alpha, Q = _proposal_case(M=300, seed=2)
    K = 700
    a = torch.from_numpy(alpha).cuda()
    q = torch.from_numpy(Q.view(np.int32)).cuda()
    i1, t1 = arsel.select_proposal_broadcast(a, q, K, seed=8, step=1, want_trials=True)
    i2, t2 = arsel.select_proposal(a.expand(K, -1).contiguous(), q.expand(K, -1).contiguous(),
                                   seed=8, step=1, want_trials=True)
    assert torch.equal(i1, i2) and torch.equal(t1, t2)
