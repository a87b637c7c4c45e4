"""The no-allocation uneven-batch call (arsel_select_ragged_noalloc, through the
C ABI) against arsel_select_ragged: bit for bit, on two calls in a row with
the second batch smaller than the first, then against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1404_0027_amd import arsel, workloads
from tests.parity import assert_same, same_float_bits

pytestmark = pytest.mark.gpu


def _both(rb, *, seed, step, t_max=4096):
    a = torch.from_numpy(np.ascontiguousarray(rb.alpha, np.float32)).cuda()
    off = torch.from_numpy(np.ascontiguousarray(rb.offsets, np.int64)).cuda()
    K = off.numel() - 1
    ri, ra, rt = arsel.select_ragged(a, off, seed=seed, step=step, t_max=t_max,
                                     want_alpha0=True, want_trials=True)
    ni = torch.full((K,), -99, dtype=torch.int32, device="cuda")
    na = torch.full((K,), -99.0, dtype=torch.float32, device="cuda")
    nt = torch.full((K,), -99, dtype=torch.int32, device="cuda")
    arsel.select_ragged_noalloc(a, off, seed=seed, step=step, t_max=t_max, index=ni, alpha0=na,
                                trials=nt)
    torch.cuda.synchronize()
    ref = (ri.cpu().numpy(), ra.cpu().numpy(), rt.cpu().numpy().view(np.uint32))
    got = (ni.cpu().numpy(), na.cpu().numpy(), nt.cpu().numpy().view(np.uint32))
    return got, ref


def _check(got, ref, what):
    assert np.array_equal(got[0], ref[0]), f"{what}: index differs at {np.nonzero(got[0] != ref[0])[0][:10]}"
    assert np.array_equal(got[2], ref[2]), f"{what}: trials differ"
    assert same_float_bits(got[1], ref[1]), f"{what}: alpha0 differs"


def test_noalloc_matches_ragged_two_calls(gpu):
    big = workloads.ragged_mix(K=3000, seed=71, log2_lo=0, log2_hi=15)
    small = workloads.ragged_mix(K=700, seed=72, log2_lo=0, log2_hi=13)
    got, ref = _both(big, seed=5, step=1)
    _check(got, ref, "first call (K=3000)")
    got2, ref2 = _both(small, seed=5, step=2)
    _check(got2, ref2, "second call (K=700)")
    o = oracle.select_ragged(small.alpha, small.offsets, seed=5, step=2, t_max=4096, threads=8)
    assert_same(got2, o, "second call vs oracle")


def test_noalloc_fallback_and_edge_sizes(gpu):
    rb = workloads.ragged_mix(K=257, seed=73, log2_lo=0, log2_hi=14)
    sizes = np.diff(rb.offsets)
    sizes[[0, 17, 200]] = 0          # empty instances report -1
    off = np.zeros(sizes.size + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    alpha = np.concatenate([rb.alpha[rb.offsets[k]:rb.offsets[k] + sizes[k]]
                            for k in range(sizes.size)]).astype(np.float32)
    rb2 = workloads.RaggedBatch(alpha=alpha, offsets=off, family=rb.family)
    for t_max in (0, 130):
        got, ref = _both(rb2, seed=8, step=t_max, t_max=t_max)
        _check(got, ref, f"t_max={t_max}")
        assert np.all(got[0][[0, 17, 200]] == -1)


def test_noalloc_hard_rows_in_pieces(gpu):
    """Heavy-tailed rows of up to ~185000 elements are hard; with pieces of
    2048 floats and at most 32 chunks per row the longest rows' chunks are
    tested piece by piece, with budgets that send most of them to the
    fallback."""
    s0 = arsel.get_schedule()
    try:
        arsel.set_schedule(arsel.Schedule(256, 8, 2048, 1))
        rng = np.random.default_rng(74)
        sizes = np.round(2 ** rng.uniform(9, 17.5, 80)).astype(np.int64)
        off = np.zeros(81, np.int64)
        np.cumsum(sizes, out=off[1:])
        alpha = rng.lognormal(0.0, 3.0, int(off[-1])).astype(np.float32)
        rb = workloads.RaggedBatch(alpha=alpha, offsets=off, family=np.full(80, 2, np.int8))
        for t_max in (0, 3, 4096):
            got, ref = _both(rb, seed=9, step=t_max, t_max=t_max)
            _check(got, ref, f"t_max={t_max}")
            o = oracle.select_ragged(alpha, off, seed=9, step=t_max, t_max=t_max, threads=8)
            assert_same(got, o, f"t_max={t_max} vs oracle")
    finally:
        arsel.set_schedule(s0)


def test_noalloc_huge_instance(gpu):
    """One instance of 2^24 + 7 reactions: 32 chunks of several LDS pieces each."""
    rng = np.random.default_rng(23)
    sizes = np.array([5, (1 << 24) + 7, 100], np.int64)
    off = np.zeros(4, np.int64)
    np.cumsum(sizes, out=off[1:])
    alpha = rng.lognormal(0, 2, int(off[-1])).astype(np.float32)
    rb = workloads.RaggedBatch(alpha=alpha, offsets=off, family=np.full(3, 2, np.int8))
    for t_max in (4096, 0):
        got, ref = _both(rb, seed=4, step=t_max, t_max=t_max)
        _check(got, ref, f"t_max={t_max}")
        o = oracle.select_ragged(alpha, off, seed=4, step=t_max, t_max=t_max, threads=8)
        assert_same(got, o, f"t_max={t_max} vs oracle")


def test_noalloc_rejects_oversized_batch(gpu):
    K = arsel.RAGGED_NOALLOC_MAX_K + 1
    a = torch.ones(K, dtype=torch.float32, device="cuda")
    off = torch.arange(K + 1, dtype=torch.int64, device="cuda")
    idx = torch.empty(K, dtype=torch.int32, device="cuda")
    with pytest.raises(arsel.ArselError, match=r"\(-2\)"):
        arsel.select_ragged_noalloc(a, off, seed=1, index=idx)
