"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs (propensity vectors, ragged batches, reaction
networks, species counts).  It holds none of the selection method's
arithmetic, so both the HIP path and the CPU oracle may consume its output.

Workloads (the paper validates on discrete Gaussians and on the propensity
vector of a 641-species / 1029-reaction yeast iron model, section
"Test and validation of the algorithm"; that vector is not public, so the
skewed families below stand in for it):

* ``uniform_vector``   - M values U(0,1], one vector broadcast to K instances.
* ``lognormal_soa``    - K realizations x M reactions, lognormal(0, 2) with a
  Bernoulli(0.3) mask set exactly to zero, stored SoA ``a[j*K + k]``.
* ``ragged_mix``       - instances with M = round(2**U(6,16)), one family per
  instance among U(0,1], Exp(1), lognormal(0,3); AoS with int64 offsets.
* ``gaussian_vector``  - the paper's discrete Gaussian test vector.
* ``mass_action_network`` / ``poisson_counts`` - a synthetic mass-action
  network (1-2 reactants per reaction, rate constants lognormal(0,2)) and
  Poisson(50) species counts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def uniform_vector(M: int = 16, seed: int = 1) -> np.ndarray:
    """M propensities U(0,1] (1 - U[0,1)), float32."""
    rng = np.random.default_rng(seed)
    return (1.0 - rng.random(M)).astype(np.float32)


def lognormal_soa(M: int = 1029, K: int = 4096, seed: int = 2, buffers: int = 1,
                  sigma: float = 2.0, zero_frac: float = 0.3) -> np.ndarray:
    """``buffers`` independent SoA batches, shape [buffers, M, K], float32.

    Entry (b, j, k) is reaction j of realization k in batch b.  Each entry is
    lognormal(0, sigma), then set exactly to zero with probability zero_frac.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((buffers, M, K), dtype=np.float32)
    for b in range(buffers):
        a = rng.lognormal(0.0, sigma, size=(M, K)).astype(np.float32)
        a[rng.random((M, K)) < zero_frac] = 0.0
        out[b] = a
    return out


@dataclass
class RaggedBatch:
    alpha: np.ndarray    # float32, concatenated instances
    offsets: np.ndarray  # int64 [K+1]
    family: np.ndarray   # int8 [K]: 0 U(0,1], 1 Exp(1), 2 lognormal(0,3)

    @property
    def K(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)


def ragged_mix(K: int = 10000, seed: int = 3, log2_lo: float = 6.0,
               log2_hi: float = 16.0) -> RaggedBatch:
    """K instances, M_k = round(2**U(log2_lo, log2_hi)), one family each."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(2.0 ** rng.uniform(log2_lo, log2_hi, size=K)).astype(np.int64)
    sizes = np.maximum(sizes, 1)
    family = rng.integers(0, 3, size=K).astype(np.int8)
    offsets = np.zeros(K + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    alpha = np.empty(int(offsets[-1]), dtype=np.float32)
    for f in range(3):
        idx = np.nonzero(family == f)[0]
        n = int(sizes[idx].sum())
        if f == 0:
            vals = 1.0 - rng.random(n)
        elif f == 1:
            vals = rng.exponential(1.0, size=n)
        else:
            vals = rng.lognormal(0.0, 3.0, size=n)
        vals = vals.astype(np.float32)
        pos = 0
        for k in idx:
            m = int(sizes[k])
            alpha[offsets[k]:offsets[k] + m] = vals[pos:pos + m]
            pos += m
    return RaggedBatch(alpha=alpha, offsets=offsets, family=family)


def gaussian_vector(M: int) -> np.ndarray:
    """The paper's discrete Gaussian: x_j = -5 + 10 j/(M-1), 1e5 * N(0,1) density."""
    x = -5.0 + np.arange(M, dtype=np.float64) * (10.0 / (M - 1))
    dens = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return (1e5 * dens).astype(np.float32)


@dataclass
class Network:
    """Mass-action network.  Reaction j consumes species r0[j] (and r1[j] when
    r1[j] >= 0) and produces p0[j] (and p1[j] when p1[j] >= 0).  A reaction
    has as many products as reactants, so the molecule count is conserved."""
    N: int
    r0: np.ndarray   # int32 [M]
    r1: np.ndarray   # int32 [M], -1 when unimolecular
    p0: np.ndarray   # int32 [M]
    p1: np.ndarray   # int32 [M], -1 when unimolecular
    rate: np.ndarray  # float32 [M]

    @property
    def M(self) -> int:
        return int(self.r0.shape[0])


def mass_action_network(N: int = 641, M: int = 1029, seed: int = 4) -> Network:
    rng = np.random.default_rng(seed)
    order = rng.integers(1, 3, size=M)             # 1 or 2 reactants, p = 1/2
    r0 = rng.integers(0, N, size=M).astype(np.int32)
    r1 = rng.integers(0, N, size=M).astype(np.int32)
    p0 = rng.integers(0, N, size=M).astype(np.int32)
    p1 = rng.integers(0, N, size=M).astype(np.int32)
    r1[order == 1] = -1
    p1[order == 1] = -1
    rate = rng.lognormal(0.0, 2.0, size=M).astype(np.float32)
    return Network(N=N, r0=r0, r1=r1, p0=p0, p1=p1, rate=rate)


def poisson_counts(N: int = 641, R: int = 1, lam: float = 50.0, seed: int = 5) -> np.ndarray:
    """Species counts, int32 [R, N], Poisson(lam)."""
    rng = np.random.default_rng(seed)
    return rng.poisson(lam, size=(R, N)).astype(np.int32)
