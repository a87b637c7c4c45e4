"""Pins of the oracle's SSA time step tau = ln(1/u) / alpha_0 (section "The
Stochastic Simulation Algorithm"), in the arithmetic both sides fix:

- -ln u by Tang's table-driven method (ACM TOMS 16(4), 1990) is checked
  against a 50-digit decimal logarithm;
- alpha_0 (128-bit fixed-point sum at the scale 2^E, rounded once) is the
  exact rational sum rounded to nearest when the propensities lie within
  104 - ceil(log2 M) binades of 2^E, independent of their order, scales by
  powers of two, and stays within its truncation bound below that range;
- the run's times: every step adds -ln u / alpha_0 with u from word 0 of
  Philox block 0xFFFFFFFE of the tag-2 stream and alpha_0 the step state's
  exact propensity sum rounded once.
"""
import dataclasses
import math
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1404_0027_amd import workloads

TAU_BLOCK = 0xFFFFFFFE


def _exact_neg_ln(w: int) -> Decimal:
    getcontext().prec = 50
    return -(Decimal(2 * w + 1) / Decimal(2 ** 33)).ln()


def _ulps(v: float, ex: Decimal) -> float:
    return float(abs(Decimal(v) - ex) / Decimal(math.ulp(float(ex))))


def test_neg_ln_against_decimal_log():
    rng = np.random.default_rng(12)
    special = [0, 1, 2, 3, 2 ** 31 - 1, 2 ** 31, 2 ** 32 - 1, 2 ** 32 - 2,
               3 * 2 ** 30, 3 * 2 ** 30 - 1, 3 * 2 ** 29]
    # u near 1 (c = 1, e = 0: the result is log1p(r) alone, where a wrong
    # polynomial term shows), near the breakpoints m = (i + 1/2) / 128, and
    # spread over all exponents
    near_one = list(rng.integers(int(2 ** 32 * (1 - 2 ** -8)), 2 ** 32, 3000))
    mids = [int((i + 0.5) / 128 * 2 ** 32) + d for i in range(96, 128) for d in (-1, 0, 1)]
    spread = list((rng.random(3000) * 2.0 ** rng.integers(0, 33, 3000)).astype(np.int64)
                  .clip(0, 2 ** 32 - 1))
    ws = special + near_one + mids + spread
    worst = max(_ulps(oracle.neg_ln_uniform(int(w)), _exact_neg_ln(int(w))) for w in ws)
    assert worst <= 2.0, worst
    # exact closed form at the smallest u: -ln 2^-33 (u = 2^-33 exactly)
    assert _ulps(oracle.neg_ln_uniform(0), Decimal(33) * Decimal(2).ln()) <= 1.0


def test_neg_ln_is_monotone_and_positive():
    ws = np.concatenate([np.arange(0, 5000), np.arange(2 ** 31 - 2500, 2 ** 31 + 2500),
                         np.arange(2 ** 32 - 5000, 2 ** 32)])
    v = np.array([oracle.neg_ln_uniform(int(w)) for w in ws])
    assert np.all(v > 0)
    assert np.all(np.diff(v) <= 0)          # u grows with w, -ln u falls


def _exact_sum(a) -> Fraction:
    return sum((Fraction(float(x)) for x in a if 0 < x < np.inf), Fraction(0))


def _log_uniform(rng, M, lo, hi):
    return (2.0 ** rng.uniform(lo, hi, M)).astype(np.float32)


@pytest.mark.parametrize("M,lo,hi", [(1, -3, 3), (7, -20, 20), (100, -40, 30),
                                     (1029, -60, 10), (5000, -120, -100),
                                     (300, 100, 127.9)])
def test_alpha0_is_the_exact_sum_rounded_once(M, lo, hi):
    rng = np.random.default_rng(M)
    a = _log_uniform(rng, M, lo, hi)
    a[rng.random(M) < 0.2] = 0.0
    a[0] = max(a[0], np.float32(2.0 ** lo))
    E = oracle.exponent_above(a.max())
    assert oracle.wide_alpha0(a, E) == float(_exact_sum(a))


def test_alpha0_of_subnormals_and_the_largest_float():
    sub = np.array([1e-45, 3e-44, 1.1e-38, 0.0, 7e-40], np.float32)
    E = oracle.exponent_above(sub.max())
    assert oracle.wide_alpha0(sub, E) == float(_exact_sum(sub))
    big = np.full(1000, np.finfo(np.float32).max, np.float32)
    assert oracle.exponent_above(big[0]) == 128
    assert oracle.wide_alpha0(big, 128) == float(_exact_sum(big))


def test_alpha0_ignores_invalid_and_nonpositive_entries():
    a = np.array([1.5, -2.0, np.nan, np.inf, -0.0, 0.25], np.float32)
    assert oracle.wide_alpha0(a, 1) == 1.75


def test_alpha0_is_order_free_and_scales_by_powers_of_two():
    rng = np.random.default_rng(3)
    a = _log_uniform(rng, 777, -100, 20)       # beyond the exact range: truncation
    E = oracle.exponent_above(a.max())
    v = oracle.wide_alpha0(a, E)
    for _ in range(3):
        assert oracle.wide_alpha0(rng.permutation(a), E) == v
    for k in (-7, 1, 50):
        assert oracle.wide_alpha0(a * np.float32(2.0 ** k), E + k) == v * 2.0 ** k


@pytest.mark.parametrize("extra", [0, 5, 40])
def test_alpha0_truncation_bound(extra):
    # a scale above the maximum (a stale envelope between exact steps) and
    # values spread beyond the exact range: the parts below 2^-sh are
    # dropped, so the result sits at most M 2^-sh (plus one rounding) below
    # the exact sum
    rng = np.random.default_rng(extra + 1)
    M = 2000
    a = _log_uniform(rng, M, -140, 10)
    E = oracle.exponent_above(a.max()) + extra
    sh = 127 - (M - 1).bit_length() - E
    v = Fraction(oracle.wide_alpha0(a, E))
    ex = _exact_sum(a)
    half_ulp = Fraction(math.ulp(float(ex))) / 2
    assert ex - M * Fraction(2) ** -sh - half_ulp <= v <= ex + half_ulp


def _stoich_apply(net, x, j):
    x[net.r0[j]] -= 1
    if net.r1[j] >= 0:
        x[net.r1[j]] -= 1
    x[net.p0[j]] += 1
    if net.p1[j] >= 0:
        x[net.p1[j]] += 1


def rated_network(kind: str):
    """The 24-species, 40-reaction test network with its own rates or with
    rates spread over 60 binades, near FLT_MAX / 5000 (alpha_max at 2^127 ..
    2^128, so the scale exponent reaches 128), or subnormal (every
    propensity subnormal)."""
    net = workloads.mass_action_network(N=24, M=40, seed=9)
    rng = np.random.default_rng(5)
    if kind == "spread":
        rate = 2.0 ** rng.uniform(-45, 15, 40)
    elif kind == "huge":
        rate = 5e34 * rng.uniform(0.5, 1.0, 40)
    elif kind == "subnormal":
        rate = 2e-44 * rng.integers(1, 4, 40)
    else:
        return net
    return dataclasses.replace(net, rate=rate.astype(np.float32))


@pytest.mark.parametrize("kind", ["network", "spread", "huge", "subnormal"])
@pytest.mark.parametrize("period", [1, 7])
def test_run_times_step_by_step(period, kind):
    """Every recorded time is the previous one plus -ln u / alpha_0, rebuilt
    from the pinned parts: the state from the fired reactions, alpha_0 as the
    exact sum of that state's propensities rounded once, u from the pinned
    Philox stream.  With rates spread over 60 binades the binary64 sum in
    index order differs from the exact one at most steps; the other rate
    sets take the scale to both ends of the float range."""
    net = rated_network(kind)
    X0 = workloads.poisson_counts(N=24, R=3, seed=2)
    ids = np.array([0, 5, 77], np.uint32)
    seed, step0, steps = 17, 3, 60
    _, t, fired, times = oracle.ssa_run(net, X0, seed=seed, step0=step0, steps=steps, ids=ids,
                                        want_times=True, period=period)
    assert (fired >= 0).mean() > 0.9
    for r in range(3):
        x = X0[r].copy()
        prev = 0.0
        for i in range(steps):
            j = int(fired[i, r])
            if j >= 0:
                a = oracle.propensities(net, x[None, :])[0]
                w = oracle.draw(seed, TAU_BLOCK, int(ids[r]), step0 + i, oracle.TAG_SSA)[0]
                expect = prev + oracle.neg_ln_uniform(int(w)) / float(_exact_sum(a))
                assert times[i, r] == expect, (r, i)
                _stoich_apply(net, x, j)
            else:
                assert times[i, r] == prev
            prev = times[i, r]
        assert t[r] == prev


def _collapse_net():
    # species A, B, C; A -> C at rate 2^60 fires first (with probability
    # 1 - 1e-31), then B -> C and C -> B run with propensities near 2^-47
    i32 = lambda v: np.array(v, np.int32)
    return workloads.Network(N=3, r0=i32([0, 1, 2]), r1=i32([-1, -1, -1]), p0=i32([2, 2, 1]),
                             p1=i32([-1, -1, -1]),
                             rate=np.array([2.0 ** 60, 1.2345e-15, 1.3e-15], np.float32))


@pytest.mark.parametrize("period", [1, 64])
def test_scale_is_taken_again_after_a_collapse(period):
    """After the 2^60 propensity collapses, the sum at the old scale (E = 61,
    sh = 64) keeps only about 17 bits of the propensities near 2^-47; it is
    below 2^(95-L), so the next step that fires takes the scale from its own
    alpha_max and alpha_0 is again the exact sum rounded once.  Without that
    rule most of these steps would differ from the exact sum."""
    net = _collapse_net()
    X0 = np.tile(np.array([[1, 5, 0]], np.int32), (4, 1))
    seed, step0, steps = 5, 1, 100
    _, _, fired, times = oracle.ssa_run(net, X0, seed=seed, step0=step0, steps=steps,
                                        want_times=True, period=period)
    assert np.all(fired[0] == 0)
    stale_differs = 0
    for r in range(4):
        x = X0[r].copy()
        prev = 0.0
        for i in range(steps):
            j = int(fired[i, r])
            assert j >= 0
            a = oracle.propensities(net, x[None, :])[0]
            w = oracle.draw(seed, TAU_BLOCK, r, step0 + i, oracle.TAG_SSA)[0]
            exact = _exact_sum(a)
            stale = sum(math.floor(Fraction(float(v)) * 2 ** 64) for v in a) / Fraction(2 ** 64)
            stale_differs += i > 0 and float(stale) != float(exact)
            assert times[i, r] == prev + oracle.neg_ln_uniform(int(w)) / float(exact), (r, i)
            prev = times[i, r]
            _stoich_apply(net, x, j)
    assert stale_differs > 100
