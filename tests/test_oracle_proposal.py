"""Pins of the oracle's proposal selector: whatever the integer proposal Q,
the output law is the exact law of oracle/laws.py, which equals
alpha_j / alpha_0 up to the 32-bit u grid; the per-trial acceptance is
alpha_0 / (c+ sum Q) up to the same grid."""
import numpy as np

import oracle
from oracle import laws
from paper_1404_0027_amd import workloads


def _quantise(q, alpha, L):
    Q = np.floor(q * 2.0 ** (31 - L)).astype(np.uint64)
    Q = np.maximum(Q, 1)
    Q[alpha <= 0] = 0
    return Q.astype(np.uint32)


def _run(alpha, Q, steps=40, K=2000, seed=3):
    M = alpha.shape[0]
    A = np.broadcast_to(alpha, (K, M))
    QQ = np.broadcast_to(Q, (K, M))
    counts = np.zeros(M)
    tsum = 0
    for s in range(steps):
        idx, tr = oracle.select_proposal(A, QQ, seed=seed, step=s, threads=8)
        assert np.all(idx >= 0)
        counts += np.bincount(idx, minlength=M)
        tsum += int(tr.sum())
    return counts, tsum / counts.sum()


def test_proposal_exact_for_random_and_adversarial_q():
    rng = np.random.default_rng(21)
    M = 200
    alpha = rng.lognormal(0, 2, size=M).astype(np.float32)
    alpha[rng.random(M) < 0.3] = 0
    L = laws.ceil_log2(M)
    exact = alpha.astype(np.float64) / alpha.astype(np.float64).sum()
    sup = alpha > 0
    # a good q (close to alpha), a random q, and one that prefers the small
    # propensities (adversarial)
    q_good = exact * rng.uniform(0.7, 1.3, size=M)
    q_rand = rng.random(M) * sup
    q_adv = np.where(sup, 1.0 / np.maximum(alpha, 1e-30), 0.0)
    for q in (q_good, q_rand, q_adv):
        q = q / q.sum()
        Q = _quantise(q, alpha, L)
        law, acc = laws.proposal_law(alpha, Q, 4096)
        # each acceptance probability is alpha_j / (c+ Q_j) rounded to the
        # 2^-32 grid: weight w_j = q_j A_j / 2^32 is off by at most q_j 2^-32,
        # their sum (= acc) by at most 2^-32, so P(j) = w_j / sum w is off by
        # at most (q_j + P(j)) 2^-32 / acc
        qn = Q.astype(np.float64) / Q.astype(np.float64).sum()
        bound = (qn + exact) * 2.0 ** -32 / acc * 1.01 + 1e-13
        assert np.all(np.abs(law - exact) <= bound)
        counts, mean_trials = _run(alpha, Q)
        assert np.all(counts[~sup] == 0)
        assert laws.chi_square_p(counts, law) > 0.01
        # closed-form acceptance: alpha_0 / (c+ sum Q)
        cplus = float(laws.proposal_cplus(alpha, Q))
        acc_cf = float(alpha.astype(np.float64).sum()) / (cplus * float(Q.astype(np.float64).sum()))
        assert abs(acc - acc_cf) / acc_cf < 1e-4
        if acc > 0.01:
            assert abs(mean_trials - 1.0 / acc) < 0.05 / acc


def test_proposal_uniform_q_equals_uniform_law():
    """Q_j = 1 on every j is the uniform proposal; its law is the exact law of
    the uniform selector for the same alpha (different random streams)."""
    a = workloads.uniform_vector(16, seed=1)
    Q = np.ones(16, np.uint32)
    law_p, acc_p = laws.proposal_law(a, Q, 4096)
    law_u = laws.uniform_law(a, 4096)
    assert np.max(np.abs(law_p - law_u) / law_u) < 1e-6


def test_proposal_invalid_cases():
    a = np.array([1.0, 0.0, 2.0], np.float32)
    bad_support = np.array([[1, 5, 0]], np.uint32)         # alpha_2 > 0 but Q_2 = 0
    idx, _ = oracle.select_proposal(a[None], bad_support, seed=1)
    assert idx[0] == -4
    too_big = np.array([[1 << 31, 0, 1 << 31]], np.uint32)  # sum Q = 2^32
    idx, _ = oracle.select_proposal(a[None], too_big, seed=1)
    assert idx[0] == -4
    idx, _ = oracle.select_proposal(np.zeros((1, 3), np.float32), np.ones((1, 3), np.uint32),
                                    seed=1)
    assert idx[0] == -1
    idx, _ = oracle.select_proposal(np.array([[1.0, np.nan, 1.0]], np.float32),
                                    np.ones((1, 3), np.uint32), seed=1)
    assert idx[0] == -2


def test_proposal_fallback_matches_uniform_fallback():
    """Both selectors share the same inverse-transform rule; with t_max = 0 the
    proposal's answer is that rule on its own (tag 1) random stream."""
    rng = np.random.default_rng(4)
    M, K = 300, 64
    a = rng.exponential(1.0, size=(K, M)).astype(np.float32)
    Q = np.ones((K, M), np.uint32)
    idx, tr = oracle.select_proposal(a, Q, seed=8, step=2, t_max=0)
    assert np.all(tr == 1)
    for k in range(K):
        F, shift = laws.fixed_weights(a[k])
        P = np.cumsum(np.array(F, dtype=np.uint64), dtype=np.uint64)
        w = oracle.draw(8, 0xFFFFFFFF, k, 2, oracle.TAG_PROPOSAL)
        V = int(w[0]) | (int(w[1]) << 32)
        target = (V * int(P[-1])) >> 64
        assert idx[k] == int(np.searchsorted(P, np.uint64(target), side="right"))
