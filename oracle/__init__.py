"""CPU oracle for the acceptance-rejection selector -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  The product (``paper_1404_0027_amd``) never does, and
this package never imports the product: the two share no code.

``arsel_oracle.c`` holds the plain sequential algorithms (Philox4x32-10,
uniform and proposal acceptance-rejection with the exact inverse-transform
fallback, mass-action propensities, the SSA jump chain); this module wraps
them with ctypes and numpy arrays.  ``laws.py`` holds closed forms used to
pin them; ``mlp.py`` the numpy forward/backward of the learned proposal.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "arsel_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-shared", "-fPIC", "-Wall", "-Wextra"]


def build() -> str:
    """Compile the oracle library with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, u32, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox4x32_10.restype = None
        L.orc_select_uniform.argtypes = [P, i64, i64, i64, i32, P, u64, u64, u32, u32, P, P, P, i32]
        L.orc_select_uniform.restype = i32
        L.orc_select_ragged.argtypes = [P, P, i64, P, u64, u64, u32, P, P, P, i32]
        L.orc_select_ragged.restype = i32
        L.orc_select_proposal.argtypes = [P, P, i64, i64, i64, i64, u64, u64, u32, P, P, i32]
        L.orc_select_proposal.restype = i32
        L.orc_propensities.argtypes = [P, i64, i64, i64, P, P, P, P]
        L.orc_propensities.restype = None
        L.orc_ssa_chain.argtypes = [P, i64, i64, i64, P, P, P, P, P, u64, u64, i64, u32, i64,
                                    P, P, i32]
        L.orc_ssa_chain.restype = i32
        L.orc_ssa_run.argtypes = [P, i64, i64, i64, P, P, P, P, P, u32, P, u64, u64, i64, u32, P,
                                  P, P, i32]
        L.orc_ssa_run.restype = i32
        L.orc_select_paper.argtypes = [P, i64, i64, i64, ctypes.c_double, u64, u64, P, i32]
        L.orc_select_paper.restype = i32
        L.orc_select_ids.argtypes = [P, i64, i64, P, u64, u64, u32, P, P, P, i32]
        L.orc_select_ids.restype = i32
        L.orc_ssa_run_proposal.argtypes = [P, i64, i64, i64, P, P, P, P, P, P, i64, u32, u32, P,
                                           u64, u64, i64, u32, P, P, P, i32]
        L.orc_ssa_run_proposal.restype = i32
        L.orc_neg_ln_uniform.argtypes = [u32]
        L.orc_neg_ln_uniform.restype = ctypes.c_double
        L.orc_wide_alpha0.argtypes = [P, i64, i32]
        L.orc_wide_alpha0.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


AOS, SOA = 0, 1
DEBUG_CHECK_BOUND = 1
TAG_UNIFORM, TAG_PROPOSAL, TAG_SSA = 0, 1, 2
FALLBACK_WORD = 0xFFFFFFFF


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one counter (4 x u32) under one key (2 x u32)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw(seed: int, word0: int, inst: int, step: int, tag: int) -> np.ndarray:
    """The four words of one trial: counter (word0, inst, step lo, step hi ^ tag<<28)."""
    ctr = [word0 & 0xFFFFFFFF, inst & 0xFFFFFFFF, step & 0xFFFFFFFF,
           ((step >> 32) ^ (tag << 28)) & 0xFFFFFFFF]
    return philox(ctr, [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])


def select_uniform(alpha: np.ndarray, M: int, K: int, ld: int, layout: int = AOS, *,
                   seed: int, step: int = 0, t_max: int = 4096, bound=None, flags: int = 0,
                   want_alpha0: bool = True, want_trials: bool = True, threads: int = 1):
    """Sequential uniform AR for K instances.  Returns (index, alpha0, trials)."""
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    b = None if bound is None else np.ascontiguousarray(bound, dtype=np.float32)
    idx = np.empty(K, dtype=np.int32)
    a0 = np.empty(K, dtype=np.float32) if want_alpha0 else None
    tr = np.empty(K, dtype=np.uint32) if want_trials else None
    rc = lib().orc_select_uniform(_p(a), M, K, ld, layout, _p(b), seed, step, t_max, flags,
                                  _p(idx), _p(a0), _p(tr), threads)
    if rc != 0:
        raise ValueError(f"orc_select_uniform rejected its arguments ({rc})")
    return idx, a0, tr


def select_ragged(alpha: np.ndarray, offsets: np.ndarray, *, seed: int, step: int = 0,
                  t_max: int = 4096, want_alpha0: bool = True, want_trials: bool = True,
                  ids=None, threads: int = 1):
    """Instance k = alpha[offsets[k]:offsets[k+1]]; with ids, only those instances
    (outputs in the order of ids)."""
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    sel = None if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
    n = off.shape[0] - 1 if sel is None else sel.shape[0]
    idx = np.empty(n, dtype=np.int32)
    a0 = np.empty(n, dtype=np.float32) if want_alpha0 else None
    tr = np.empty(n, dtype=np.uint32) if want_trials else None
    rc = lib().orc_select_ragged(_p(a), _p(off), n, _p(sel), seed, step, t_max, _p(idx),
                                 _p(a0), _p(tr), threads)
    if rc != 0:
        raise ValueError("orc_select_ragged rejected its arguments")
    return idx, a0, tr


def select_proposal(alpha: np.ndarray, Q: np.ndarray, *, seed: int, step: int = 0,
                    t_max: int = 4096, threads: int = 1):
    """alpha float32 [K, M], Q uint32 [K, M].  Returns (index, trials)."""
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    q = np.ascontiguousarray(Q, dtype=np.uint32)
    K, M = a.shape
    idx = np.empty(K, dtype=np.int32)
    tr = np.empty(K, dtype=np.uint32)
    rc = lib().orc_select_proposal(_p(a), _p(q), M, K, M, M, seed, step, t_max, _p(idx),
                                   _p(tr), threads)
    if rc != 0:
        raise ValueError("orc_select_proposal rejected its arguments")
    return idx, tr


def select_proposal_broadcast(alpha: np.ndarray, Q: np.ndarray, K: int, *, seed: int,
                              step: int = 0, t_max: int = 4096, threads: int = 1):
    """K instances sharing one alpha [M] and one Q [M] (instance k keeps its
    own stream).  Returns (index, trials)."""
    a = np.ascontiguousarray(alpha, dtype=np.float32).ravel()
    q = np.ascontiguousarray(Q, dtype=np.uint32).ravel()
    M = a.shape[0]
    idx = np.empty(K, dtype=np.int32)
    tr = np.empty(K, dtype=np.uint32)
    rc = lib().orc_select_proposal(_p(a), _p(q), M, K, 0, 0, seed, step, t_max, _p(idx),
                                   _p(tr), threads)
    if rc != 0:
        raise ValueError("orc_select_proposal rejected its arguments")
    return idx, tr


def propensities(net, X: np.ndarray) -> np.ndarray:
    """Mass-action propensities alpha[r, j] of states X[r, i] (int32)."""
    x = np.ascontiguousarray(X, dtype=np.int32)
    R, N = x.shape
    M = int(net.r0.shape[0])
    out = np.empty((R, M), dtype=np.float32)
    lib().orc_propensities(_p(x), R, N, M, _p(np.ascontiguousarray(net.r0, np.int32)),
                           _p(np.ascontiguousarray(net.r1, np.int32)),
                           _p(np.ascontiguousarray(net.rate, np.float32)), _p(out))
    return out


def ssa_chain(net, X0: np.ndarray, *, seed: int, step0: int, steps: int, t_max: int = 4096,
              rec_from: int | None = None, threads: int = 1):
    """Run the jump chain.  Returns (X_final, recorded states or None, fired[steps, R])."""
    x = np.array(X0, dtype=np.int32, copy=True, order="C")
    R, N = x.shape
    M = int(net.r0.shape[0])
    rec = None
    if rec_from is not None:
        rec = np.empty((steps - rec_from, R, N), dtype=np.int32)
    fired = np.empty((steps, R), dtype=np.int32)
    arrs = [np.ascontiguousarray(v, np.int32) for v in (net.r0, net.r1, net.p0, net.p1)]
    rate = np.ascontiguousarray(net.rate, np.float32)
    lib().orc_ssa_chain(_p(x), R, N, M, *[_p(v) for v in arrs], _p(rate), seed, step0, steps,
                        t_max, 0 if rec_from is None else rec_from, _p(rec), _p(fired), threads)
    return x, rec, fired


def ssa_run(net, X0: np.ndarray, *, seed: int, step0: int, steps: int, t_max: int = 4096,
            t0=None, ids=None, want_times: bool = False, threads: int = 1, Q=None,
            qfloor: int = 1, period: int = 1):
    """Full SSA run (direct method with the AR selection and the time step);
    with Q ([R, M] uint32) the proposal AR selects, with
    Q'_j = max(Q_j, qfloor, 1).  period p: the envelopes are exact at the
    call's first step and at steps s with s mod p = 0, running maxima between.
    Returns (X_final, t_final float64 [R], fired [steps, R], times or None)."""
    x = np.array(X0, dtype=np.int32, copy=True, order="C")
    R, N = x.shape
    M = int(net.r0.shape[0])
    t = np.zeros(R, np.float64) if t0 is None else np.array(t0, np.float64, copy=True)
    fired = np.empty((steps, R), dtype=np.int32)
    times = np.empty((steps, R), dtype=np.float64) if want_times else None
    idv = None if ids is None else np.ascontiguousarray(ids, np.uint32)
    arrs = [np.ascontiguousarray(v, np.int32) for v in (net.r0, net.r1, net.p0, net.p1)]
    rate = np.ascontiguousarray(net.rate, np.float32)
    if Q is None:
        lib().orc_ssa_run(_p(x), R, N, M, *[_p(v) for v in arrs], _p(rate), period, _p(idv), seed,
                          step0, steps, t_max, _p(t), _p(times), _p(fired), threads)
    else:
        q = np.ascontiguousarray(Q, dtype=np.uint32)
        lib().orc_ssa_run_proposal(_p(x), R, N, M, *[_p(v) for v in arrs], _p(rate), _p(q), M,
                                   qfloor, period, _p(idv), seed, step0, steps, t_max, _p(t),
                                   _p(times), _p(fired), threads)
    return x, t, fired, times


def neg_ln_uniform(w: int) -> float:
    """-ln u of the SSA time step for u = (w + 1/2) 2^-32 (Tang's table-driven ln)."""
    return float(lib().orc_neg_ln_uniform(int(w) & 0xFFFFFFFF))


def wide_alpha0(alpha, E: int) -> float:
    """alpha_0 of the SSA time step: sum of floor(alpha_j 2^sh) over the finite
    positive alpha_j, sh = 127 - ceil(log2 M) - E, rounded once to binary64 and
    scaled back by 2^-sh."""
    a = np.ascontiguousarray(alpha, dtype=np.float32).ravel()
    return float(lib().orc_wide_alpha0(_p(a), a.shape[0], int(E)))


def exponent_above(x: float) -> int:
    """E with 2^(E-1) <= x < 2^E for a finite x > 0."""
    return int(np.frexp(np.float32(x))[1])


PAPER_REJECT = -5


def select_paper(alpha: np.ndarray, M: int, K: int, ld: int, *, w: float = 1.0, seed: int,
                 step: int = 0, threads: int = 1) -> np.ndarray:
    """The paper's election/selection scheme for K instances (alpha[k*ld + j],
    ld = 0 broadcasts).  Returns index int32 [K] (-5: election failed)."""
    a = np.ascontiguousarray(alpha, dtype=np.float32)
    idx = np.empty(K, dtype=np.int32)
    rc = lib().orc_select_paper(_p(a), M, K, ld, float(w), seed, step, _p(idx), threads)
    if rc != 0:
        raise ValueError("orc_select_paper rejected its arguments")
    return idx


def select_ids(rows: np.ndarray, ids, *, seed: int, step: int = 0, t_max: int = 4096,
               threads: int = 1):
    """Uniform AR on rows [n, M] that are instances ids[i] of a larger batch.
    Returns (index, alpha0, trials)."""
    a = np.ascontiguousarray(rows, dtype=np.float32)
    n, M = a.shape
    idv = np.ascontiguousarray(ids, np.uint32)
    idx = np.empty(n, np.int32)
    a0 = np.empty(n, np.float32)
    tr = np.empty(n, np.uint32)
    rc = lib().orc_select_ids(_p(a), M, n, _p(idv), seed, step, t_max, _p(idx), _p(a0), _p(tr),
                              threads)
    if rc != 0:
        raise ValueError("orc_select_ids rejected its arguments")
    return idx, a0, tr
