"""Pins of the oracle's uniform acceptance-rejection selector.

What fixes the answers here is not the oracle itself:
  * the exact output law (oracle/laws.py, an enumeration over the 32-bit u
    grid) and chi-square tests against it and against alpha_j / alpha_0
    (the SSA's selection law, section "The Stochastic Simulation Algorithm");
  * an independent numpy inverse transform for the fallback;
  * special cases with a forced answer and bit-exact invariants.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import laws
from paper_1404_0027_amd import workloads


def _trial_words(seed, t, k, step, tag=0):
    """Trial t uses Philox block t // 2: words (0, 1) for even t, (2, 3) for odd."""
    w = oracle.draw(seed, t >> 1, k, step, tag)
    h = t & 1
    return int(w[2 * h]), int(w[2 * h + 1])


def _lemire_reference(seed, k, step, M, t_max, tag=0):
    """Candidate of the first trial whose Lemire draw is not rejected, by
    Python integer arithmetic on Philox words."""
    thr = (1 << 32) % M
    for t in range(t_max):
        cw, _ = _trial_words(seed, t, k, step, tag)
        m = cw * M
        if (m & 0xFFFFFFFF) >= thr:
            return m >> 32, t + 1
    return None, None


def test_lemire_fold_rule_exhaustive_16bit():
    """The folded rejection rule gives exactly floor(2^B / M) preimages per
    candidate, checked exhaustively at B = 16 for every M < 600."""
    B = 16
    w = np.arange(1 << B, dtype=np.int64)
    for M in range(1, 600):
        m = w * M
        keep = (m & ((1 << B) - 1)) >= ((1 << B) % M)
        counts = np.bincount((m >> B)[keep], minlength=M)
        assert counts.shape[0] == M
        assert np.all(counts == (1 << B) // M), M


def test_all_equal_is_first_unrejected_candidate():
    """With every alpha_j equal, fl64((1-2^-32) a) < a, so every trial that
    survives the candidate draw accepts."""
    M, K = 1029, 300
    a = np.full(M, 3.5, dtype=np.float32)
    idx, a0, tr = oracle.select_uniform(a, M, K, 0, seed=77, step=5)
    for k in range(K):
        j, t = _lemire_reference(77, k, 5, M, 4096)
        assert idx[k] == j and tr[k] == t


def test_lemire_rejections_are_skipped():
    """M = 3,000,017 has 2^32 mod M / 2^32 ~ 5e-4, so some of 8000 instances
    see a rejected first draw; the oracle must skip exactly those."""
    M, K = 3_000_017, 8000
    a = np.ones(M, dtype=np.float32)
    idx, _, tr = oracle.select_uniform(a, M, K, 0, seed=3, step=0, want_alpha0=False,
                                       threads=8)
    assert (tr > 1).sum() > 0
    for k in np.nonzero(tr > 1)[0][:20].tolist() + list(range(50)):
        j, t = _lemire_reference(3, k, 0, M, 4096)
        assert idx[k] == j and tr[k] == t


def test_trial_sequence_brute_force():
    """Replay the trial sequence with Python integers and exact rationals:
    candidate j = floor(c M / 2^32) unless Lemire rejects; u = v / 2^32;
    accept iff u * alpha_max < alpha_j, decided exactly (the binary64 product
    of a 32-bit u and a 24-bit alpha_max is exact)."""
    from fractions import Fraction

    a = np.array([0.5, 0.0, 2.0, 1.25, 0.03125, 3.0, 0.75, 1.5], np.float32)
    M, K = 8, 400
    idx, _, tr = oracle.select_uniform(a, M, K, 0, seed=123, step=77)
    amax = Fraction(float(a.max()))
    for k in range(K):
        for t in range(4096):
            cw, uw = _trial_words(123, t, k, 77, 0)
            m = cw * M
            if (m & 0xFFFFFFFF) < (1 << 32) % M:
                continue
            j = m >> 32
            u = Fraction(uw, 1 << 32)
            if u * amax < Fraction(float(a[j])):
                break
        assert idx[k] == j and tr[k] == t + 1, k


def test_special_cases():
    s = dict(seed=1, step=0)
    # M = 1
    idx, a0, tr = oracle.select_uniform(np.array([2.0], np.float32), 1, 5, 0, **s)
    assert np.all(idx == 0) and np.all(a0 == 2.0)
    # a single nonzero
    a = np.zeros(64, np.float32)
    a[37] = 1e-3
    idx, a0, _ = oracle.select_uniform(a, 64, 50, 0, **s)
    assert np.all(idx == 37) and np.all(a0 == np.float32(1e-3))
    # all zero
    idx, a0, tr = oracle.select_uniform(np.zeros(10, np.float32), 10, 4, 0, **s)
    assert np.all(idx == -1) and np.all(a0 == 0) and np.all(tr == 0)
    # invalid entries
    for bad in (np.nan, -1.0, np.inf, -np.inf):
        a = np.ones(10, np.float32)
        a[3] = bad
        idx, a0, _ = oracle.select_uniform(a, 10, 3, 0, **s)
        assert np.all(idx == -2) and np.all(np.isnan(a0))
    # -0.0 is a zero propensity, not a negative one
    a = np.array([-0.0, 1.0], np.float32)
    idx, _, _ = oracle.select_uniform(a, 2, 20, 0, **s)
    assert np.all(idx == 1)


def test_fallback_matches_numpy_inverse_transform():
    """t_max = 0 forces the fixed-point inverse transform for every instance;
    recompute it independently: F_j = floor(alpha_j 2^(63-L-E)) in float64,
    integer prefixes, target = floor(V S / 2^64), searchsorted."""
    rng = np.random.default_rng(5)
    for M in (1, 2, 3, 7, 64, 1029, 5000):
        K = 40
        alpha = rng.lognormal(0, 3, size=(K, M)).astype(np.float32)
        alpha[rng.random((K, M)) < 0.3] = 0
        alpha[:, 0] = np.maximum(alpha[:, 0], 1e-30)   # keep every row non-zero
        idx, a0, tr = oracle.select_uniform(alpha, M, K, M, seed=99, step=1234, t_max=0)
        assert np.all(tr == 1)
        for k in range(K):
            row = alpha[k].astype(np.float64)
            _, E = math.frexp(row.max())
            L = laws.ceil_log2(M)
            F = np.floor(np.ldexp(row, 63 - L - E)).astype(np.uint64)
            P = np.cumsum(F, dtype=np.uint64)
            S = int(P[-1])
            assert 0 < S < (1 << 63)
            w = oracle.draw(99, 0xFFFFFFFF, k, 1234, 0)
            V = int(w[0]) | (int(w[1]) << 32)
            target = (V * S) >> 64
            j = int(np.searchsorted(P, np.uint64(target), side="right"))
            assert idx[k] == j
            assert a0[k] == np.float32(math.ldexp(float(np.float32(S)), -(63 - L - E)))


def test_fallback_law_is_fixed_point_proportional():
    """Over many steps the forced fallback samples F_j / S (chi-square)."""
    a = workloads.uniform_vector(16, seed=1)
    K, steps = 1024, 100
    counts = np.zeros(16)
    for s in range(steps):
        idx, _, _ = oracle.select_uniform(a, 16, K, 0, seed=1, step=s, t_max=0,
                                          want_alpha0=False, want_trials=False)
        counts += np.bincount(idx, minlength=16)
    F, _ = laws.fixed_weights(a)
    p = np.array(F, dtype=np.float64) / sum(F)
    assert laws.chi_square_p(counts, p) > 0.01


def test_chi_square_config1():
    """M=16 U(0,1], K=1024, seed 1, steps 0..999: 1.024e6 selections pass a
    chi-square test against the exact law and against alpha_j / alpha_0."""
    a = workloads.uniform_vector(16, seed=1)
    K = 1024
    counts = np.zeros(16)
    trials_sum = 0
    for s in range(1000):
        idx, _, tr = oracle.select_uniform(a, 16, K, 0, seed=1, step=s, want_alpha0=False)
        counts += np.bincount(idx, minlength=16)
        trials_sum += int(tr.sum())
    law = laws.uniform_law(a, 4096)
    exact = a.astype(np.float64) / a.astype(np.float64).sum()
    assert np.max(np.abs(law - exact) / exact) < 1e-6
    assert laws.chi_square_p(counts, law) > 0.01
    assert laws.chi_square_p(counts, exact) > 0.01
    # mean trials of a geometric law with the closed-form per-trial acceptance
    acc = laws.per_trial_acceptance(a)
    mean = trials_sum / counts.sum()
    assert abs(mean - 1.0 / acc) < 0.01 * (1.0 / acc)


def test_chi_square_skewed_lognormal():
    """One lognormal(0,2) vector with 30% zeros (the batched workload's
    distribution), 2e5 selections, against the exact law."""
    a = workloads.lognormal_soa(M=1029, K=1, seed=2)[0, :, 0].copy()
    K = 2000
    counts = np.zeros(1029)
    for s in range(100):
        idx, _, _ = oracle.select_uniform(a, 1029, K, 0, seed=7, step=s, want_alpha0=False,
                                          want_trials=False, threads=8)
        counts += np.bincount(idx, minlength=1029)
    law = laws.uniform_law(a, 4096)
    assert np.all(counts[a == 0] == 0)
    assert laws.chi_square_p(counts, law) > 0.01


def test_scaling_by_power_of_two_is_bit_identical():
    rng = np.random.default_rng(8)
    M, K = 333, 200
    a = rng.lognormal(0, 2, size=(K, M)).astype(np.float32)
    a[rng.random((K, M)) < 0.3] = 0
    base = oracle.select_uniform(a, M, K, M, seed=4, step=9)
    for e in (-20, -1, 3, 40):
        s = oracle.select_uniform(np.ldexp(a, e).astype(np.float32), M, K, M, seed=4, step=9)
        assert np.array_equal(base[0], s[0]) and np.array_equal(base[2], s[2])
        assert np.array_equal(np.ldexp(base[1], e).astype(np.float32), s[1])
    # forced fallback scales the same way
    b0 = oracle.select_uniform(a, M, K, M, seed=4, step=9, t_max=0)
    b1 = oracle.select_uniform(np.ldexp(a, 17).astype(np.float32), M, K, M, seed=4, step=9,
                               t_max=0)
    assert np.array_equal(b0[0], b1[0])


def test_subnormal_vector_law():
    """Subnormal float propensities are ordinary numbers in the binary64
    product, so the maximal entries still always accept and the law holds."""
    a = np.full(8, np.float32(3e-44), dtype=np.float32)   # subnormal in float32
    a[2] = np.float32(7e-45)
    A = laws.accept_counts(a, float(a.max()))
    assert A[0] == laws.GRID
    counts = np.zeros(8)
    for s in range(40):
        idx, _, _ = oracle.select_uniform(a, 8, 2000, 0, seed=2, step=s, want_alpha0=False,
                                          want_trials=False)
        counts += np.bincount(idx, minlength=8)
    assert laws.chi_square_p(counts, laws.uniform_law(a, 4096)) > 0.01


def test_layouts_agree():
    """AoS rows, SoA columns and a padded leading dimension select the same."""
    rng = np.random.default_rng(12)
    M, K = 97, 130
    a = rng.exponential(1.0, size=(K, M)).astype(np.float32)
    aos = oracle.select_uniform(a, M, K, M, oracle.AOS, seed=5, step=2)
    soa_buf = np.zeros((M, K + 3), np.float32)
    soa_buf[:, :K] = a.T
    soa = oracle.select_uniform(soa_buf, M, K, K + 3, oracle.SOA, seed=5, step=2)
    for x, y in zip(aos, soa):
        assert np.array_equal(x, y)


def test_supplied_bound():
    """Any bound >= max is exact (the law only scales the acceptance); a bound
    below the true max is reported as -3 in debug mode."""
    rng = np.random.default_rng(13)
    M, K = 50, 4000
    a = rng.random(M).astype(np.float32)
    bound = np.full(K, np.float32(a.max() * 3), np.float32)
    counts = np.zeros(M)
    for s in range(10):
        idx, _, tr = oracle.select_uniform(a, M, K, 0, seed=6, step=s, bound=bound,
                                           want_alpha0=False)
        counts += np.bincount(idx, minlength=M)
    assert laws.chi_square_p(counts, laws.uniform_law(a, 4096, env=float(bound[0]))) > 0.01
    small = np.full(K, np.float32(a.max() / 2), np.float32)
    idx, _, _ = oracle.select_uniform(a, M, K, 0, seed=6, bound=small,
                                      flags=oracle.DEBUG_CHECK_BOUND)
    assert np.all(idx == -3)
    idx, _, _ = oracle.select_uniform(a, M, 4, 0, seed=6,
                                      bound=np.array([0, -1, np.nan, np.inf], np.float32))
    assert list(idx) == [-1, -2, -2, -2]


def test_ragged_matches_dense():
    rb = workloads.ragged_mix(K=60, seed=3, log2_lo=0, log2_hi=10)
    idx, a0, tr = oracle.select_ragged(rb.alpha, rb.offsets, seed=10, step=3)
    for k in range(rb.K):
        lo, hi = rb.offsets[k], rb.offsets[k + 1]
        # a dense call with one instance at id 0 would use counter k = 0, so
        # compare through a K-instance broadcast call and take instance k
        d = oracle.select_uniform(rb.alpha[lo:hi], int(hi - lo), k + 1, 0, seed=10, step=3)
        assert (idx[k], a0[k], tr[k]) == (d[0][k], d[1][k], d[2][k])


def test_threads_do_not_change_results():
    a = workloads.lognormal_soa(M=1029, K=512, seed=2)[0]
    r1 = oracle.select_uniform(a, 1029, 512, 512, oracle.SOA, seed=1, step=4, threads=1)
    r8 = oracle.select_uniform(a, 1029, 512, 512, oracle.SOA, seed=1, step=4, threads=8)
    for x, y in zip(r1, r8):
        assert np.array_equal(x, y)


def test_select_ids_matches_the_batch():
    """Rows checked by instance id give the batch's answers for those ids."""
    a = workloads.lognormal_soa(M=300, K=200, seed=2)[0]
    i, a0, t = oracle.select_uniform(a, 300, 200, 200, oracle.SOA, seed=4, step=3)
    ids = np.array([0, 17, 199, 5], np.uint32)
    i2, a02, t2 = oracle.select_ids(a[:, ids].T, ids, seed=4, step=3)
    assert np.array_equal(i[ids], i2) and np.array_equal(t[ids], t2)
    assert np.array_equal(a0[ids].view(np.uint32), a02.view(np.uint32))
