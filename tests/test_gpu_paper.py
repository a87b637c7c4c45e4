"""GPU parity of the paper's own election/selection scheme against the CPU
oracle, bit for bit, and its law (the closed form of oracle/laws.py)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import laws
from paper_1404_0027_amd import arsel, workloads

pytestmark = pytest.mark.gpu


def _both(alpha, M, K, ld, *, w, seed, step):
    g = arsel.select_paper(torch.from_numpy(np.ascontiguousarray(alpha, np.float32)).cuda(), M, K,
                           ld, w=w, seed=seed, step=step).cpu().numpy()
    o = oracle.select_paper(alpha, M, K, ld, w=w, seed=seed, step=step, threads=8)
    return g, o


@pytest.mark.parametrize("M", [64, 256, 1024])
@pytest.mark.parametrize("w", [1.0, 0.5, 2.0])
def test_paper_broadcast_gaussian(gpu, M, w):
    g, o = _both(workloads.gaussian_vector(M), M, 5000, 0, w=w, seed=3, step=M)
    assert np.array_equal(g, o)


def test_paper_rejections(gpu):
    # M = 2, w = 2: the election fails with probability 5/12
    g, o = _both(np.array([1.0, 3.0], np.float32), 2, 4000, 0, w=2.0, seed=6, step=1)
    assert np.array_equal(g, o)
    assert 1400 < (g == arsel.PAPER_REJECT).sum() < 1950


def test_paper_aos_rows_and_statuses(gpu):
    rng = np.random.default_rng(4)
    K, M, ld = 777, 1029, 1040
    a = rng.lognormal(0.0, 2.0, (K, ld)).astype(np.float32)
    a[rng.random((K, ld)) < 0.3] = 0.0
    a[0, :] = 0.0                      # -1
    a[1, 17] = np.nan                  # -2
    a[2, 3] = -1.0                     # -2
    a[3, :M] = 0.0
    a[3, 5] = -0.0                     # still all zero: -1
    a[4, :M] = 0.0
    a[4, 9] = 1e-40                    # one subnormal propensity
    g, o = _both(a, M, K, ld, w=1.0, seed=9, step=2)
    assert np.array_equal(g, o)
    assert g[0] == -1 and g[1] == -2 and g[2] == -2 and g[3] == -1 and g[4] == 9


def test_paper_large_rows(gpu):
    rng = np.random.default_rng(5)
    M, K = 70001, 6
    a = rng.exponential(1.0, (K, M)).astype(np.float32)
    g, o = _both(a, M, K, M, w=1.0, seed=1, step=8)
    assert np.array_equal(g, o)


def test_paper_law_on_gpu(gpu):
    a = workloads.gaussian_vector(64)
    t = torch.from_numpy(a).cuda()
    counts = np.zeros(64)
    for s in range(16):
        idx = arsel.select_paper(t, 64, 65536, 0, w=1.0, seed=7, step=s)
        counts += np.bincount(idx.cpu().numpy(), minlength=64)
    law, _ = laws.paper_law(a.astype(np.float64), 1.0)
    assert laws.chi_square_p(counts, law) > 0.01
    assert laws.chi_square_p(counts, a / a.sum()) < 1e-6
