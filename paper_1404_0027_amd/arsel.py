"""Python binding of libarsel.so (ctypes; argument marshalling only).

Every step of the selection runs in the library's HIP kernels.  PyTorch is
used for device memory and streams: tensors in, tensors out, launched on the
current torch stream.  If the library is missing this module raises; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libarsel.so")

AOS, SOA = 0, 1
DEBUG_CHECK_BOUND = 1
TAG_UNIFORM, TAG_PROPOSAL, TAG_SSA = 0, 1, 2


class ArselError(RuntimeError):
    pass


_lib = None
_lock = threading.Lock()
_ctx: dict[int, ctypes.c_void_p] = {}


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ArselError(f"{LIB_PATH} is not built; run `python -m paper_1404_0027_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_uint32, ctypes.c_uint64)
        L.arsel_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
        L.arsel_create.restype = ctypes.c_int
        L.arsel_destroy.argtypes = [P]
        L.arsel_destroy.restype = ctypes.c_int
        L.arsel_strerror.argtypes = [ctypes.c_int]
        L.arsel_strerror.restype = ctypes.c_char_p
        L.arsel_select.argtypes = [P, P, i32, i32, i64, ctypes.c_int, P, u64, u64, u32, u32,
                                   P, P, P, P]
        L.arsel_select.restype = ctypes.c_int
        for name, argtypes in _EXTRA_SIGNATURES.items():
            fn = getattr(L, name, None)
            if fn is not None:
                fn.argtypes = argtypes
                fn.restype = ctypes.c_int
        _lib = L
    return _lib


class Schedule(ctypes.Structure):
    _fields_ = [("wave_max_m", ctypes.c_int32), ("block_waves", ctypes.c_int32),
                ("lds_max_m", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class Network(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("r0", ctypes.c_void_p),
                ("r1", ctypes.c_void_p), ("p0", ctypes.c_void_p), ("p1", ctypes.c_void_p),
                ("rate", ctypes.c_void_p)]


class MLP(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("M", ctypes.c_int32), ("H", ctypes.c_int32),
                ("Kp", ctypes.c_int32), ("Mp", ctypes.c_int32), ("W1", ctypes.c_void_p),
                ("W2", ctypes.c_void_p), ("W3", ctypes.c_void_p), ("b1", ctypes.c_void_p),
                ("b2", ctypes.c_void_p), ("b3", ctypes.c_void_p)]


class MLPTrain(ctypes.Structure):
    _fields_ = [("net", MLP), ("master", ctypes.c_void_p * 6), ("grad", ctypes.c_void_p * 6),
                ("m", ctypes.c_void_p * 6), ("v", ctypes.c_void_p * 6),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_P = ctypes.c_void_p
_EXTRA_SIGNATURES = {
    "arsel_select_proposal": [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                              ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                              _P, _P, _P],
    "arsel_propensities": [_P, ctypes.POINTER(Network), _P, ctypes.c_int32, _P, _P],
    "arsel_ssa_chain": [_P, ctypes.POINTER(Network), _P, ctypes.c_int32, ctypes.c_uint64,
                        ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int64, _P, _P,
                        _P],
    "arsel_mlp_forward": [_P, ctypes.POINTER(MLP), _P, ctypes.c_int32, _P, _P, _P, _P],
    "arsel_mlp_train_step": [_P, ctypes.POINTER(MLPTrain), _P, _P, ctypes.c_int32, ctypes.c_float,
                             ctypes.c_int32, _P, _P],
    "arsel_mlp_sync_bf16": [_P, ctypes.POINTER(MLPTrain), _P],
    "arsel_gemm_bf16": [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_int32,
                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32, _P,
                        ctypes.c_int64, _P],
    "arsel_select_ragged": [_P, _P, _P, ctypes.c_int32, _P, ctypes.c_uint64, ctypes.c_uint64,
                            ctypes.c_uint32, _P, _P, _P, _P],
    "arsel_select_ragged_noalloc": [_P, _P, _P, ctypes.c_int32, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint32, _P, _P, _P, _P],
    "arsel_probe_read": [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                         _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _P],
    "arsel_set_mlp_fused": [_P, ctypes.c_int32],
    "arsel_get_schedule": [_P, ctypes.POINTER(Schedule)],
    "arsel_set_schedule": [_P, ctypes.POINTER(Schedule)],
    "arsel_set_dense_config": [_P, ctypes.c_int32, ctypes.c_int32],
    "arsel_set_trial_lanes": [_P, ctypes.c_int32],
    "arsel_select_paper": [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                           ctypes.c_uint64, ctypes.c_uint64, _P, _P],
    "arsel_ssa_deps": [_P, ctypes.POINTER(Network), _P, _P, _P],
    "arsel_ssa_run": [_P, ctypes.POINTER(Network), _P, _P, _P, ctypes.c_int32, ctypes.c_uint64,
                      ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, _P, _P,
                      _P, _P],
    "arsel_ssa_run_proposal": [_P, ctypes.POINTER(Network), _P, _P, _P, ctypes.c_int64,
                               ctypes.c_uint32, _P, ctypes.c_int32, ctypes.c_uint64,
                               ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                               _P, _P, _P, _P],
}

SSA_DEP_MAX = 64


def _check(rc: int, what: str) -> None:
    if rc != 0:
        msg = lib().arsel_strerror(rc).decode()
        raise ArselError(f"{what} failed ({rc}): {msg}")


def context(device: int | torch.device | None = None) -> ctypes.c_void_p:
    """The library context of a device (created once per process)."""
    if device is None:
        device = torch.cuda.current_device()
    if isinstance(device, torch.device):
        device = device.index if device.index is not None else torch.cuda.current_device()
    with _lock:
        c = _ctx.get(device)
        if c is None:
            c = ctypes.c_void_p()
            _check(lib().arsel_create(ctypes.byref(c), device), "arsel_create")
            _ctx[device] = c
    return c


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t: torch.Tensor, dtype, numel: int, name: str, device) -> None:
    if not isinstance(t, torch.Tensor) or t.dtype != dtype:
        raise ArselError(f"{name} must be a {dtype} tensor")
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ArselError(f"{name} must live on the same GPU")
    if not t.is_contiguous():
        raise ArselError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ArselError(f"{name} holds {t.numel()} elements, {numel} needed")


def select(alpha: torch.Tensor, M: int, K: int, ld: int, layout: int = AOS, *, seed: int,
           step: int = 0, t_max: int = 4096, bound: torch.Tensor | None = None, flags: int = 0,
           want_alpha0: bool = False, want_trials: bool = False,
           index: torch.Tensor | None = None, alpha0: torch.Tensor | None = None,
           trials: torch.Tensor | None = None):
    """K selections from a dense batch (see arsel_select in include/arsel.h).

    alpha: float32 CUDA tensor; AoS element (k, j) at k*ld + j (ld = 0: one
    vector for all), SoA element (k, j) at j*ld + k.  Returns
    (index int32 [K], alpha0 float32 [K] or None, trials int32 [K] or None);
    trials hold uint32 bit patterns.
    """
    dev = alpha.device
    if layout == AOS:
        need = M if ld == 0 else (K - 1) * ld + M if K > 0 else 0
    else:
        need = (M - 1) * ld + K if K > 0 else 0
    _need(alpha, torch.float32, need, "alpha", None)
    if index is None:
        index = torch.empty(K, dtype=torch.int32, device=dev)
    _need(index, torch.int32, K, "index", dev)
    if want_alpha0 and alpha0 is None:
        alpha0 = torch.empty(K, dtype=torch.float32, device=dev)
    if alpha0 is not None:
        _need(alpha0, torch.float32, K, "alpha0", dev)
    if want_trials and trials is None:
        trials = torch.empty(K, dtype=torch.int32, device=dev)
    if trials is not None:
        _need(trials, torch.int32, K, "trials", dev)
    if bound is not None:
        _need(bound, torch.float32, K, "bound", dev)
    rc = lib().arsel_select(context(dev), _ptr(alpha), M, K, ld, layout, _ptr(bound),
                            seed & (2**64 - 1), step & (2**64 - 1), t_max, flags, _ptr(index),
                            _ptr(alpha0), _ptr(trials), _stream(dev))
    _check(rc, "arsel_select")
    return index, alpha0, trials


def select_raw(ctx, alpha_ptr: int, M: int, K: int, ld: int, layout: int, bound_ptr, seed: int,
               step: int, t_max: int, flags: int, index_ptr: int, alpha0_ptr, trials_ptr,
               stream_handle: int) -> int:
    """Unchecked call with raw device pointers (for timing loops and tests of
    the host-side argument checks).  Returns the library's status code."""
    return lib().arsel_select(ctx, alpha_ptr, M, K, ld, layout, bound_ptr, seed, step, t_max,
                              flags, index_ptr, alpha0_ptr, trials_ptr, stream_handle)


def set_dense_config(tile: int, waves: int, device=None) -> None:
    """Instances per dense tile and wavefronts per workgroup (results
    unchanged); (0, 0) restores the automatic choice."""
    _check(lib().arsel_set_dense_config(context(device), tile, waves), "arsel_set_dense_config")


def set_trial_lanes(lanes: int, device=None) -> None:
    """Lanes per instance of the broadcast kernels (0: automatic; else a power
    of two in 1..64).  Results unchanged."""
    _check(lib().arsel_set_trial_lanes(context(device), lanes), "arsel_set_trial_lanes")


def get_schedule(device=None) -> Schedule:
    s = Schedule()
    _check(lib().arsel_get_schedule(context(device), ctypes.byref(s)), "arsel_get_schedule")
    return s


def set_mlp_fused(on: bool, device=None) -> None:
    """Inference forward by the fused kernel or layer by layer (the default)."""
    _check(lib().arsel_set_mlp_fused(context(device), 1 if on else 0), "arsel_set_mlp_fused")


def set_schedule(s: Schedule, device=None) -> None:
    _check(lib().arsel_set_schedule(context(device), ctypes.byref(s)), "arsel_set_schedule")


def select_ragged(alpha: torch.Tensor, offsets: torch.Tensor, *, seed: int, step: int = 0,
                  t_max: int = 4096, host_offsets=None, want_alpha0: bool = False,
                  want_trials: bool = False, index: torch.Tensor | None = None,
                  alpha0: torch.Tensor | None = None, trials: torch.Tensor | None = None):
    """Uneven batch (arsel_select_ragged): scan, split, hard chunks, pick.

    alpha: float32 CUDA tensor of concatenated instances; offsets: int64 CUDA
    tensor [K+1].  host_offsets: the same offsets as a numpy array (optional);
    when given, they are checked against alpha's size and the work lists are
    built on the host (otherwise on the device, three more small launches).
    Repeated calls with the same sizes (and schedule) reuse the work lists
    already on the device: the call is then four kernel launches.  Calls
    sharing a device context must run on one stream, since the lists and
    counters live in the context.
    """
    import numpy as np

    dev = alpha.device
    if not isinstance(offsets, torch.Tensor) or offsets.dtype != torch.int64:
        raise ArselError("offsets must be an int64 tensor")
    K = offsets.numel() - 1
    if K < 0:
        raise ArselError("offsets needs K+1 entries")
    _need(offsets, torch.int64, K + 1, "offsets", dev)
    _need(alpha, torch.float32, 0, "alpha", None)
    sizes = None
    if host_offsets is not None:
        ho = np.ascontiguousarray(host_offsets, dtype=np.int64)
        if ho.shape[0] != K + 1:
            raise ArselError("host_offsets must have K+1 entries")
        sizes = np.diff(ho)
        if K > 0 and (ho[0] < 0 or np.any(sizes < 0) or ho[-1] > alpha.numel()):
            raise ArselError("host_offsets must be non-decreasing and within alpha")
        sizes = np.ascontiguousarray(sizes, dtype=np.int64)
    if index is None:
        index = torch.empty(K, dtype=torch.int32, device=dev)
    _need(index, torch.int32, K, "index", dev)
    if want_alpha0 and alpha0 is None:
        alpha0 = torch.empty(K, dtype=torch.float32, device=dev)
    if alpha0 is not None:
        _need(alpha0, torch.float32, K, "alpha0", dev)
    if want_trials and trials is None:
        trials = torch.empty(K, dtype=torch.int32, device=dev)
    if trials is not None:
        _need(trials, torch.int32, K, "trials", dev)
    sp = None if sizes is None else sizes.ctypes.data_as(ctypes.c_void_p)
    rc = lib().arsel_select_ragged(context(dev), _ptr(alpha), _ptr(offsets), K, sp,
                                   seed & (2**64 - 1), step & (2**64 - 1), t_max, _ptr(index),
                                   _ptr(alpha0), _ptr(trials), _stream(dev))
    _check(rc, "arsel_select_ragged")
    return index, alpha0, trials


RAGGED_NOALLOC_MAX_K = 65536


def select_ragged_noalloc(alpha: torch.Tensor, offsets: torch.Tensor, *, seed: int,
                          step: int = 0, t_max: int = 4096, index: torch.Tensor,
                          alpha0: torch.Tensor | None = None,
                          trials: torch.Tensor | None = None) -> None:
    """Uneven batch without any allocation (arsel_select_ragged_noalloc).

    The caller passes every output tensor; the work lists and counters live in
    the library's static per-GPU scratch array (K <= RAGGED_NOALLOC_MAX_K).
    Calls on one GPU share that array: do not overlap them.
    """
    dev = alpha.device
    if not isinstance(offsets, torch.Tensor) or offsets.dtype != torch.int64:
        raise ArselError("offsets must be an int64 tensor")
    K = offsets.numel() - 1
    if K < 0:
        raise ArselError("offsets needs K+1 entries")
    _need(offsets, torch.int64, K + 1, "offsets", dev)
    _need(alpha, torch.float32, 0, "alpha", None)
    _need(index, torch.int32, K, "index", dev)
    if alpha0 is not None:
        _need(alpha0, torch.float32, K, "alpha0", dev)
    if trials is not None:
        _need(trials, torch.int32, K, "trials", dev)
    rc = lib().arsel_select_ragged_noalloc(context(dev), _ptr(alpha), _ptr(offsets), K,
                                           seed & (2**64 - 1), step & (2**64 - 1), t_max,
                                           _ptr(index), _ptr(alpha0), _ptr(trials), _stream(dev))
    _check(rc, "arsel_select_ragged_noalloc")


def select_proposal(alpha: torch.Tensor, Q: torch.Tensor, *, seed: int, step: int = 0,
                    t_max: int = 4096, want_trials: bool = False,
                    index: torch.Tensor | None = None, trials: torch.Tensor | None = None):
    """AR with the integer proposal Q (arsel_select_proposal).  alpha float32
    [K, M] and Q int32/uint32 bit patterns [K, M], both CUDA and contiguous."""
    if alpha.dim() != 2 or Q.shape != alpha.shape:
        raise ArselError("alpha and Q must be [K, M] tensors of the same shape")
    K, M = alpha.shape
    dev = alpha.device
    _need(alpha, torch.float32, K * M, "alpha", dev)
    if Q.dtype not in (torch.int32, torch.uint32):
        raise ArselError("Q must hold 32-bit integers")
    if not Q.is_contiguous() or Q.device != dev:
        raise ArselError("Q must be contiguous on the same GPU")
    if index is None:
        index = torch.empty(K, dtype=torch.int32, device=dev)
    _need(index, torch.int32, K, "index", dev)
    if want_trials and trials is None:
        trials = torch.empty(K, dtype=torch.int32, device=dev)
    if trials is not None:
        _need(trials, torch.int32, K, "trials", dev)
    rc = lib().arsel_select_proposal(context(dev), _ptr(alpha), _ptr(Q), M, K, M, M,
                                     seed & (2**64 - 1), step & (2**64 - 1), t_max, _ptr(index),
                                     _ptr(trials), _stream(dev))
    _check(rc, "arsel_select_proposal")
    return index, trials


def select_proposal_broadcast(alpha: torch.Tensor, Q: torch.Tensor, K: int, *, seed: int,
                              step: int = 0, t_max: int = 4096, want_trials: bool = False,
                              index: torch.Tensor | None = None,
                              trials: torch.Tensor | None = None):
    """K selections from ONE (alpha [M], Q [M]) pair (arsel_select_proposal with
    lda = ldq = 0): instance k uses the tag-1 stream of instance id k."""
    M = alpha.numel()
    dev = alpha.device
    _need(alpha, torch.float32, M, "alpha", dev)
    if Q.dtype not in (torch.int32, torch.uint32) or Q.numel() != M:
        raise ArselError("Q must hold M 32-bit integers")
    if not Q.is_contiguous() or Q.device != dev:
        raise ArselError("Q must be contiguous on the same GPU")
    if index is None:
        index = torch.empty(K, dtype=torch.int32, device=dev)
    _need(index, torch.int32, K, "index", dev)
    if want_trials and trials is None:
        trials = torch.empty(K, dtype=torch.int32, device=dev)
    if trials is not None:
        _need(trials, torch.int32, K, "trials", dev)
    rc = lib().arsel_select_proposal(context(dev), _ptr(alpha), _ptr(Q), M, K, 0, 0,
                                     seed & (2**64 - 1), step & (2**64 - 1), t_max, _ptr(index),
                                     _ptr(trials), _stream(dev))
    _check(rc, "arsel_select_proposal")
    return index, trials


PAPER_REJECT = -5


def select_paper(alpha: torch.Tensor, M: int, K: int, ld: int, *, w: float = 1.0, seed: int,
                 step: int = 0, index: torch.Tensor | None = None) -> torch.Tensor:
    """The paper's election/selection scheme (arsel_select_paper): K instances
    of alpha[k*ld + j] (ld = 0 broadcasts); -5 marks a failed election."""
    dev = alpha.device
    need = M if ld == 0 else (K - 1) * ld + M if K > 0 else 0
    _need(alpha, torch.float32, need, "alpha", dev)
    if index is None:
        index = torch.empty(K, dtype=torch.int32, device=dev)
    _need(index, torch.int32, K, "index", dev)
    rc = lib().arsel_select_paper(context(dev), _ptr(alpha), M, K, ld, float(w),
                                  seed & (2**64 - 1), step & (2**64 - 1), _ptr(index), _stream(dev))
    _check(rc, "arsel_select_paper")
    return index


def gemm_bf16(A: torch.Tensor, lda: int, a_kcontig: bool, B: torch.Tensor, ldb: int,
              b_kcontig: bool, M: int, N: int, K: int, bias=None, relu=False, C=None):
    """C[m][n] = sum_k A(m,k) B(n,k) on MFMA (see arsel_gemm_bf16)."""
    dev = A.device
    if A.dtype != torch.bfloat16 or B.dtype != torch.bfloat16:
        raise ArselError("A and B must be bfloat16")
    need_a = (M - 1) * lda + K if a_kcontig else (K - 1) * lda + M
    need_b = (N - 1) * ldb + K if b_kcontig else (K - 1) * ldb + N
    if A.numel() < need_a or B.numel() < need_b:
        raise ArselError("operand too small for the given shape")
    if C is None:
        C = torch.empty(M, N, dtype=torch.float32, device=dev)
    _need(C, torch.float32, M * N, "C", dev)
    if bias is not None:
        _need(bias, torch.float32, N, "bias", dev)
    rc = lib().arsel_gemm_bf16(context(dev), _ptr(A), lda, int(a_kcontig), _ptr(B), ldb,
                               int(b_kcontig), M, N, K, _ptr(bias), int(relu), _ptr(C), N,
                               _stream(dev))
    _check(rc, "arsel_gemm_bf16")
    return C


def probe_read(a: torch.Tensor, rows: int, cols: int, ld: int, tile: int = 0,
               sink: torch.Tensor | None = None) -> torch.Tensor:
    """Read-bandwidth probe (arsel_probe_read): reads the rows x cols float32
    matrix `a` (row stride ld) once; returns the per-workgroup sink.  Pass the
    sink of an earlier call to launch without allocating (graph capture)."""
    dev = a.device
    _need(a, torch.float32, rows * ld, "a", None)
    grid = ctypes.c_int64(0)
    rc = lib().arsel_probe_read(context(dev), None, rows, cols, ld, tile, None, 0,
                                ctypes.byref(grid), _stream(dev))
    if rc not in (0, -1, -2):
        _check(rc, "arsel_probe_read")
    if sink is None:
        sink = torch.empty(max(grid.value, 1), dtype=torch.int32, device=dev)
    rc = lib().arsel_probe_read(context(dev), _ptr(a), rows, cols, ld, tile, _ptr(sink),
                                sink.numel(), ctypes.byref(grid), _stream(dev))
    _check(rc, "arsel_probe_read")
    return sink
