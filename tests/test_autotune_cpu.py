"""Host-side checks of the autotuner's candidate space (no GPU)."""
from paper_1404_0027_amd import autotune


def test_ragged_candidates_fit_lds():
    for lds in (64 * 1024, 160 * 1024):
        cands = autotune.ragged_candidates(lds)
        assert cands
        for wave_max_m, bw, lds_max_m, bpc in cands:
            assert bw in (4, 8, 16) and 1 <= bpc <= 8
            need = bw * wave_max_m * 4 + 2048
            assert need <= lds and need * bpc <= 160 * 1024
            assert lds_max_m in (0, 4096, 8192)


def test_signature_is_stable():
    import numpy as np

    s = np.array([64, 65, 1000, 65536])
    assert autotune._signature(s) == autotune._signature(s.copy())
    assert autotune._signature(s) != autotune._signature(s[:3])
