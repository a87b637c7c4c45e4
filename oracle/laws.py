"""Closed-form output laws of the selectors -- TEST INFRASTRUCTURE ONLY.

These are exact enumerations, not samplers, and pin the oracle's sampling
code through chi-square tests and exact identities.

Uniform AR (the sequential rule of the paper's section "A GPU
acceptance-rejection algorithm (GPU/AR) for SSA"), with the readings used by
the oracle: one trial takes a 32-bit candidate word, maps it to a candidate by
Lemire's multiply-shift (rejecting the 2^32 mod M lowest remainders, so the
candidate is exactly uniform), and accepts when fl64(u * env) < alpha_j for u
on the 32-bit grid.  Per candidate j the number of grid points that accept is

    A_j = #{ v in [0, 2^32) : fl64(v 2^-32 * env) < alpha_j },

a monotone predicate in v, so it is found by binary search.  A trial accepts
(and picks j) with probability (1 - eps) / M * A_j / 2^32, eps = (2^32 mod M)
/ 2^32.  After t_max rejected trials the inverse transform of the section
"The Stochastic Simulation Algorithm" picks j with probability F_j / S in
exact fixed point.  So

    P(j) = (1 - (1-a)^T) A_j / sum A + (1-a)^T F_j / S,   a = (1-eps) sum A / (M 2^32).
"""
from __future__ import annotations

import math

import numpy as np


def ceil_log2(M: int) -> int:
    L = 0
    while (1 << L) < M:
        L += 1
    return L


GRID_BITS = 32
GRID = 1 << GRID_BITS


def _count_below(pred) -> np.ndarray:
    """Least v in [0, GRID] where the monotone predicate pred(v) is false."""
    # pred takes an int64 array of v values and returns a bool array
    probe = pred(np.zeros(1, dtype=np.int64))
    shape = probe.shape
    lo = np.zeros(shape, dtype=np.int64)
    hi = np.full(shape, GRID, dtype=np.int64)
    for _ in range(GRID_BITS + 2):
        mid = (lo + hi) // 2
        ok = pred(np.minimum(mid, GRID - 1)) & (mid < GRID)
        lo = np.where(ok, mid + 1, lo)
        hi = np.where(ok, hi, mid)
    return lo


def accept_counts(alpha: np.ndarray, env: float) -> np.ndarray:
    """A_j for every j (int64): grid points v with fl64(v 2^-32 env) < alpha_j."""
    a = np.asarray(alpha, dtype=np.float32).astype(np.float64)
    env = float(np.float32(env))

    def pred(v):
        u = v.astype(np.float64) * 2.0 ** -GRID_BITS
        return (u * env) < a

    return _count_below(pred)


def accept_counts_proposal(alpha: np.ndarray, Q: np.ndarray, cplus: float) -> np.ndarray:
    """A_j = #{v : fl64(fl64(v 2^-32 c+) Q_j) < alpha_j}."""
    a = np.asarray(alpha, dtype=np.float32).astype(np.float64)
    qd = np.asarray(Q, dtype=np.uint32).astype(np.float64)
    c = float(cplus)

    def pred(v):
        u = v.astype(np.float64) * 2.0 ** -GRID_BITS
        return ((u * c) * qd) < a

    return _count_below(pred)


def fixed_weights(alpha: np.ndarray, amax: float | None = None) -> tuple[list[int], int]:
    """F_j = floor(alpha_j 2^(63-L-E)) as Python ints (float64 ldexp is exact here)."""
    a = np.asarray(alpha, dtype=np.float32)
    M = a.shape[0]
    if amax is None:
        amax = float(a.max())
    _, E = math.frexp(float(np.float32(amax)))
    shift = 63 - ceil_log2(M) - E
    F = [int(math.floor(math.ldexp(float(x), shift))) for x in a]
    return F, shift


def uniform_law(alpha: np.ndarray, t_max: int, env: float | None = None) -> np.ndarray:
    """Exact P(j) of the uniform selector, float64."""
    a = np.asarray(alpha, dtype=np.float32)
    M = a.shape[0]
    amax = float(a.max())
    if env is None:
        env = amax
    A = accept_counts(a, env).astype(np.float64)
    eps = ((1 << 32) % M) / float(1 << 32)
    acc = (1.0 - eps) * A.sum() / (M * float(GRID))
    F, _ = fixed_weights(a, amax)
    S = float(sum(F))
    Ff = np.array([float(f) for f in F])
    miss = (1.0 - acc) ** t_max
    p = (1.0 - miss) * (A / A.sum() if A.sum() > 0 else 0.0) + miss * Ff / S
    return p


def per_trial_acceptance(alpha: np.ndarray, env: float | None = None) -> float:
    a = np.asarray(alpha, dtype=np.float32)
    M = a.shape[0]
    if env is None:
        env = float(a.max())
    A = accept_counts(a, env).astype(np.float64)
    eps = ((1 << 32) % M) / float(1 << 32)
    return (1.0 - eps) * A.sum() / (M * float(GRID))


def proposal_cplus(alpha: np.ndarray, Q: np.ndarray) -> float:
    """c+ = nextafter(max_j fl64(alpha_j / Q_j), +inf) over alpha_j > 0."""
    a = np.asarray(alpha, dtype=np.float32).astype(np.float64)
    q = np.asarray(Q, dtype=np.uint32).astype(np.float64)
    sup = a > 0
    r = a[sup] / q[sup]
    return float(np.nextafter(r.max(), np.inf))


def proposal_law(alpha: np.ndarray, Q: np.ndarray, t_max: int) -> tuple[np.ndarray, float]:
    """Exact P(j) of the proposal selector and its per-trial acceptance."""
    a = np.asarray(alpha, dtype=np.float32)
    q = np.asarray(Q, dtype=np.uint32)
    SQ = int(q.astype(np.uint64).sum())
    cplus = proposal_cplus(a, q)
    A = accept_counts_proposal(a, q, cplus).astype(np.float64)
    eps = ((1 << 32) % SQ) / float(1 << 32)
    w = q.astype(np.float64) / SQ * A / float(GRID)
    acc = (1.0 - eps) * w.sum()
    F, _ = fixed_weights(a)
    S = float(sum(F))
    Ff = np.array([float(f) for f in F])
    miss = (1.0 - acc) ** t_max
    return (1.0 - miss) * w / w.sum() + miss * Ff / S, acc


def chi_square_p(counts: np.ndarray, probs: np.ndarray, min_expected: float = 5.0) -> float:
    """Pearson chi-square p-value, merging bins whose expected count is < 5."""
    from scipy.stats import chi2

    counts = np.asarray(counts, dtype=np.float64)
    probs = np.asarray(probs, dtype=np.float64)
    n = counts.sum()
    exp = probs * n
    order = np.argsort(exp)
    obs_b, exp_b = [], []
    acc_o = acc_e = 0.0
    for i in order:
        acc_o += counts[i]
        acc_e += exp[i]
        if acc_e >= min_expected:
            obs_b.append(acc_o)
            exp_b.append(acc_e)
            acc_o = acc_e = 0.0
    if acc_e > 0 or acc_o > 0:
        if exp_b:
            obs_b[-1] += acc_o
            exp_b[-1] += acc_e
        else:
            obs_b.append(acc_o)
            exp_b.append(acc_e)
    obs_b = np.array(obs_b)
    exp_b = np.array(exp_b)
    stat = float(((obs_b - exp_b) ** 2 / exp_b).sum())
    dof = max(len(obs_b) - 1, 1)
    return float(chi2.sf(stat, dof))


def paper_law(alpha: np.ndarray, w: float = 1.0) -> tuple[np.ndarray, float]:
    """Law of the paper's election/selection scheme (continuous u), and the
    probability that the election fails.

    With d_j = alpha_j / T, T = w alpha_max, the ratings R_j = T U_j / alpha_j
    of the eligible reactions (R_j < 1) are independent and P(R_j > r) =
    1 - d_j r on [0, 1/d_j]; the least of them is j with probability
        P(j) = d_j * integral_0^min(1, 1/d_max) prod_{i != j} (1 - d_i r)_+ dr,
    and no reaction is eligible with probability prod_j (1 - d_j)_+ (zero when
    w <= 1).  The integrand is a polynomial of degree < M on the interval, so
    Gauss-Legendre with M nodes integrates it exactly (up to rounding)."""
    a = np.asarray(alpha, np.float64)
    T = w * a.max()
    d = a / T
    hi = min(1.0, 1.0 / d.max())
    n = max(8, a.size)
    x, wt = np.polynomial.legendre.leggauss(n)
    r = 0.5 * hi * (x + 1.0)
    wt = 0.5 * hi * wt
    terms = 1.0 - np.outer(r, d)                    # [nodes, M], > 0 inside the interval
    logt = np.log(np.where(d > 0, terms, 1.0))
    total = logt.sum(axis=1)
    law = np.empty(a.size)
    for j in range(a.size):
        if d[j] == 0:
            law[j] = 0.0
            continue
        law[j] = d[j] * np.sum(wt * np.exp(total - logt[:, j]))
    reject = float(np.prod(np.clip(1.0 - d, 0.0, None))) if w > 1 else 0.0
    return law, reject
