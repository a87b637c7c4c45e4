"""Pins of the oracle's mass-action propensities and SSA jump chain (the
state update X <- X + v_j of the paper's section "The Stochastic Simulation
Algorithm")."""
import numpy as np

import oracle
from paper_1404_0027_amd import workloads


def _tiny_net():
    # R0: A -> B (unimolecular), R1: A + B -> A + A, R2: A + A -> B + B (homodimer)
    return workloads.Network(N=2,
                             r0=np.array([0, 0, 0], np.int32), r1=np.array([-1, 1, 0], np.int32),
                             p0=np.array([1, 0, 1], np.int32), p1=np.array([-1, 0, 1], np.int32),
                             rate=np.array([0.5, 2.0, 0.25], np.float32))


def test_propensities_by_hand():
    net = _tiny_net()
    X = np.array([[3, 5], [1, 7], [0, 4]], np.int32)
    a = oracle.propensities(net, X)
    want = np.array([[0.5 * 3, 2.0 * 15, 0.25 * 3],      # h = 3, 3*5, 3*2/2
                     [0.5 * 1, 2.0 * 7, 0.0],            # homodimer needs two A
                     [0.0, 0.0, 0.0]], np.float32)
    assert np.array_equal(a, want)


def test_chain_conserves_and_stays_nonnegative():
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    X0 = workloads.poisson_counts(N=64, R=20, seed=5)
    X, rec, fired = oracle.ssa_chain(net, X0, seed=9, step0=0, steps=300, rec_from=0,
                                     threads=4)
    assert np.array_equal(X.sum(axis=1), X0.sum(axis=1))
    assert X.min() >= 0 and rec.min() >= 0
    # every fired reaction had a positive propensity in the state before it
    for i in range(0, 300, 17):
        a = oracle.propensities(net, rec[i])
        for r in range(20):
            j = fired[i, r]
            assert j >= 0 and a[r, j] > 0
    # replaying the recorded transitions reproduces the recorded states
    for i in range(299):
        for r in range(0, 20, 7):
            x = rec[i, r].copy()
            j = fired[i, r]
            x[net.r0[j]] -= 1
            if net.r1[j] >= 0:
                x[net.r1[j]] -= 1
            x[net.p0[j]] += 1
            if net.p1[j] >= 0:
                x[net.p1[j]] += 1
            assert np.array_equal(x, rec[i + 1, r])


def test_chain_is_deterministic_and_thread_independent():
    net = workloads.mass_action_network(N=64, M=100, seed=4)
    X0 = workloads.poisson_counts(N=64, R=16, seed=5)
    a = oracle.ssa_chain(net, X0, seed=3, step0=10, steps=50, threads=1)
    b = oracle.ssa_chain(net, X0, seed=3, step0=10, steps=50, threads=8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
    # splitting the run at any step gives the same chain (resume = seed, step)
    c1 = oracle.ssa_chain(net, X0, seed=3, step0=10, steps=20, threads=2)
    c2 = oracle.ssa_chain(net, c1[0], seed=3, step0=30, steps=30, threads=2)
    assert np.array_equal(c2[0], a[0])


def test_absorbing_state_fires_nothing():
    net = _tiny_net()
    X0 = np.array([[0, 9]], np.int32)           # no A: nothing can fire
    X, _, fired = oracle.ssa_chain(net, X0, seed=1, step0=0, steps=5)
    assert np.array_equal(X, X0) and np.all(fired == -1)
