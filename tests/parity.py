"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same inputs and compare element by element (bit-exact)."""
import numpy as np
import torch

import oracle
from paper_1404_0027_amd import arsel


def same_float_bits(a: np.ndarray, b: np.ndarray) -> bool:
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    na, nb = np.isnan(a), np.isnan(b)
    if not np.array_equal(na, nb):
        return False
    return np.array_equal(a[~na].view(np.uint32), b[~nb].view(np.uint32))


def dense_both(alpha_np, M, K, ld, layout, *, seed, step, t_max=4096, bound=None, flags=0,
               device="cuda:0"):
    a_dev = torch.from_numpy(np.ascontiguousarray(alpha_np, np.float32)).to(device)
    b_dev = None if bound is None else torch.from_numpy(np.asarray(bound, np.float32)).to(device)
    idx, a0, tr = arsel.select(a_dev, M, K, ld, layout, seed=seed, step=step, t_max=t_max,
                               bound=b_dev, flags=flags, want_alpha0=True, want_trials=True)
    torch.cuda.synchronize()
    g = (idx.cpu().numpy(), a0.cpu().numpy(), tr.cpu().numpy().view(np.uint32))
    o = oracle.select_uniform(alpha_np, M, K, ld, layout, seed=seed, step=step, t_max=t_max,
                              bound=bound, flags=flags, threads=8)
    return g, o


def assert_same(g, o, what=""):
    gi, ga, gt = g
    oi, oa, ot = o
    bad = np.nonzero(gi != oi)[0]
    assert bad.size == 0, f"{what}: index mismatch at {bad[:10]} gpu={gi[bad[:10]]} oracle={oi[bad[:10]]}"
    assert np.array_equal(gt, ot), f"{what}: trials mismatch at {np.nonzero(gt != ot)[0][:10]}"
    assert same_float_bits(ga, oa), f"{what}: alpha0 mismatch"
