"""Pin the oracle's Philox4x32-10 to two independent source implementations
that ship in this image: PyTorch's ATen/core/PhiloxRNGEngine.h and rocRAND's
rocrand_philox4x32_10.h (both header-only; compiled here for the host)."""
import os
import subprocess

import numpy as np
import pytest
import torch

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _grid(n=300, seed=11):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, 1 << 32, size=(n, 6), dtype=np.uint64)
    rows[:, 3] &= (1 << 30) - 1            # rocRAND's offset is 4*counter, keep it < 2^64
    fixed = np.array([[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0],
                      [0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF],
                      [1, 0, 0xFFFFFFFF, 7, 3, 0x20000000]], dtype=np.uint64)
    return np.concatenate([fixed, rows]).astype(np.uint64)


def _run(exe, grid):
    txt = "\n".join(" ".join("%x" % int(v) for v in row) for row in grid) + "\n"
    out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
    return np.array([[int(w, 16) for w in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


@pytest.fixture(scope="module")
def kat_exes(tmp_path_factory):
    d = tmp_path_factory.mktemp("kat")
    tinc = os.path.join(os.path.dirname(torch.__file__), "include")
    t_exe = str(d / "philox_torch")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", tinc, "-o", t_exe,
                    os.path.join(HERE, "kat", "philox_torch.cpp")], check=True)
    r_exe = str(d / "philox_rocrand")
    subprocess.run(["/opt/rocm/bin/hipcc", "-std=c++17", "-O1", "-o", r_exe,
                    os.path.join(HERE, "kat", "philox_rocrand.cpp")], check=True)
    return t_exe, r_exe


def test_philox_matches_torch_and_rocrand(kat_exes):
    grid = _grid()
    ref_t = _run(kat_exes[0], grid)
    ref_r = _run(kat_exes[1], grid)
    assert np.array_equal(ref_t, ref_r), "the two reference implementations disagree"
    mine = np.array([oracle.philox(row[2:6], row[0:2]) for row in grid], dtype=np.uint64)
    assert np.array_equal(mine, ref_t)


def test_philox_counter_layout():
    # draw() puts (word0, instance, step lo, step hi ^ tag<<28) in the counter
    w = oracle.draw(seed=(5 << 32) | 9, word0=3, inst=7, step=(2 << 32) | 11, tag=1)
    ref = oracle.philox([3, 7, 11, 2 ^ (1 << 28)], [9, 5])
    assert np.array_equal(w, ref)
