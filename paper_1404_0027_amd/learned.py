"""The learned proposal: training data from the SSA jump chain, a BF16 MLP
trained on the GPU by the library's own forward/backward kernels, and
selection with its quantised proposal.  All arithmetic runs in libarsel's
kernels; this module only owns tensors and calls the C ABI."""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import arsel
from .arsel import ArselError, _check, _ptr, _stream, context, lib


class DeviceNetwork:
    """A mass-action network (workloads.Network) resident on the GPU."""

    def __init__(self, net, device="cuda:0"):
        for name in ("r0", "r1", "p0", "p1"):
            v = np.asarray(getattr(net, name))
            lo = -1 if name in ("r1", "p1") else 0
            if v.shape[0] != net.M or v.min() < lo or v.max() >= net.N:
                raise ArselError(f"network array {name} out of range")
        self.N, self.M = int(net.N), int(net.M)
        self.device = torch.device(device)
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(self.device, dt)
        self.r0, self.r1 = t(net.r0, torch.int32), t(net.r1, torch.int32)
        self.p0, self.p1 = t(net.p0, torch.int32), t(net.p1, torch.int32)
        self.rate = t(net.rate, torch.float32)
        self.c = arsel.Network(self.N, self.M, self.r0.data_ptr(), self.r1.data_ptr(),
                               self.p0.data_ptr(), self.p1.data_ptr(), self.rate.data_ptr())

    def propensities(self, X: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        R = X.shape[0]
        arsel._need(X, torch.int32, R * self.N, "X", self.device)
        if out is None:
            out = torch.empty(R, self.M, dtype=torch.float32, device=self.device)
        arsel._need(out, torch.float32, R * self.M, "alpha", self.device)
        rc = lib().arsel_propensities(context(self.device), ctypes.byref(self.c), _ptr(X), R,
                                      _ptr(out), _stream(self.device))
        _check(rc, "arsel_propensities")
        return out

    def chain(self, X: torch.Tensor, *, seed: int, step0: int, steps: int, t_max: int = 4096,
              record_from: int | None = None, want_fired: bool = False):
        """Run the jump chain in place on X [R, N]; returns (recorded states
        [steps - record_from, R, N] or None, fired [steps, R] or None)."""
        R = X.shape[0]
        arsel._need(X, torch.int32, R * self.N, "X", self.device)
        rec = None
        if record_from is not None:
            rec = torch.empty(steps - record_from, R, self.N, dtype=torch.int32, device=self.device)
        fired = torch.empty(steps, R, dtype=torch.int32, device=self.device) if want_fired else None
        rc = lib().arsel_ssa_chain(context(self.device), ctypes.byref(self.c), _ptr(X), R,
                                   seed & (2**64 - 1), step0 & (2**64 - 1), steps, t_max,
                                   0 if record_from is None else record_from, _ptr(rec),
                                   _ptr(fired), _stream(self.device))
        _check(rc, "arsel_ssa_chain")
        return rec, fired


    def deps(self):
        """Dependency graph of the full run (built once on the device)."""
        if getattr(self, "_deps", None) is None:
            d = torch.empty(self.M, arsel.SSA_DEP_MAX, dtype=torch.int32, device=self.device)
            n = torch.empty(self.M, dtype=torch.int32, device=self.device)
            rc = lib().arsel_ssa_deps(context(self.device), ctypes.byref(self.c), _ptr(d), _ptr(n),
                                      _stream(self.device))
            _check(rc, "arsel_ssa_deps")
            self._deps = (d, n)
        return self._deps

    def run(self, X: torch.Tensor, t: torch.Tensor, *, seed: int, step0: int, steps: int,
            t_max: int = 4096, want_fired: bool = False, want_times: bool = False, Q=None,
            qfloor: int = 1, period: int = 1):
        """Full SSA run in place on X [R, N] (int32) and t [R] (float64);
        with Q ([R, ldq] int32/uint32 proposal, ldq >= M) the steps select
        with the proposal Q' = max(Q, qfloor, 1).  Pass qfloor on the scale of
        Q: about sum(Q) / (8 M) (for this module's network output,
        2^(31 - ceil(log2 M)) // (8 M)); with 1, a reaction inactive when Q was
        computed that turns active weighs 1 against sum(Q) and can push every
        step into the fallback.  period: envelopes exact at the first step and
        at steps s with s mod period = 0, maintained from the changed
        propensities between (64 is a good choice; 1 is exact every step).
        Returns (fired [steps, R] or None, times [steps, R] or None)."""
        R = X.shape[0]
        arsel._need(X, torch.int32, R * self.N, "X", self.device)
        arsel._need(t, torch.float64, R, "t", self.device)
        d, n = self.deps()
        fired = torch.empty(steps, R, dtype=torch.int32, device=self.device) if want_fired else None
        times = torch.empty(steps, R, dtype=torch.float64, device=self.device) if want_times else None
        common = (_ptr(X), R, seed & (2**64 - 1), step0 & (2**64 - 1), steps, t_max, period,
                  _ptr(t), _ptr(times), _ptr(fired), _stream(self.device))
        if Q is None:
            rc = lib().arsel_ssa_run(context(self.device), ctypes.byref(self.c), _ptr(d), _ptr(n),
                                     *common)
            _check(rc, "arsel_ssa_run")
        else:
            if Q.dim() != 2 or Q.shape[0] != R or Q.shape[1] < self.M:
                raise arsel.ArselError("Q must be [R, ldq] with ldq >= M")
            if Q.dtype not in (torch.int32, torch.uint32):
                raise arsel.ArselError("Q must be int32 or uint32")
            arsel._need(Q, Q.dtype, Q.numel(), "Q", self.device)
            rc = lib().arsel_ssa_run_proposal(context(self.device), ctypes.byref(self.c), _ptr(d),
                                              _ptr(n), _ptr(Q), Q.shape[1], qfloor, *common)
            _check(rc, "arsel_ssa_run_proposal")
        return fired, times


def _round_up(x: int, m: int) -> int:
    return (x + m - 1) // m * m


class LearnedProposal:
    """BF16 MLP N -> H -> H -> M with FP32 masters and Adam state on the GPU."""

    def __init__(self, N: int, M: int, H: int = 256, seed: int = 0, device="cuda:0",
                 beta1=0.9, beta2=0.999, eps=1e-8):
        self.device = torch.device(device)
        self.N, self.M, self.H = N, M, H
        self.Kp, self.Mp = _round_up(N, 32), _round_up(M, 16)
        rng = np.random.default_rng(seed)
        W1 = rng.normal(0.0, math.sqrt(2.0 / N), (H, self.Kp))
        W1[:, N:] = 0.0
        W2 = rng.normal(0.0, math.sqrt(2.0 / H), (H, H))
        W3 = rng.normal(0.0, math.sqrt(1.0 / H), (self.Mp, H))
        W3[M:] = 0.0
        shapes = [(H, self.Kp), (H,), (H, H), (H,), (self.Mp, H), (self.Mp,)]
        init = [W1, np.zeros(H), W2, np.zeros(H), W3, np.zeros(self.Mp)]
        f32 = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(self.device)
        self.master = [f32(a) for a in init]
        self.grad = [torch.zeros(s, dtype=torch.float32, device=self.device) for s in shapes]
        self.m = [torch.zeros(s, dtype=torch.float32, device=self.device) for s in shapes]
        self.v = [torch.zeros(s, dtype=torch.float32, device=self.device) for s in shapes]
        self.Wb = [torch.empty(shapes[i], dtype=torch.bfloat16, device=self.device) for i in (0, 2, 4)]
        self.t = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        net = arsel.MLP(N, M, H, self.Kp, self.Mp, self.Wb[0].data_ptr(), self.Wb[1].data_ptr(),
                        self.Wb[2].data_ptr(), self.master[1].data_ptr(),
                        self.master[3].data_ptr(), self.master[5].data_ptr())
        arr = lambda ts: (ctypes.c_void_p * 6)(*[t.data_ptr() for t in ts])
        self.c = arsel.MLPTrain(net, arr(self.master), arr(self.grad), arr(self.m), arr(self.v),
                                beta1, beta2, eps)
        self.sync()

    def sync(self) -> None:
        _check(lib().arsel_mlp_sync_bf16(context(self.device), ctypes.byref(self.c),
                                         _stream(self.device)), "arsel_mlp_sync_bf16")

    def train_step(self, X: torch.Tensor, alpha: torch.Tensor, lr: float) -> torch.Tensor:
        B = X.shape[0]
        arsel._need(X, torch.int32, B * self.N, "X", self.device)
        arsel._need(alpha, torch.float32, B * self.M, "alpha", self.device)
        self.t += 1
        rc = lib().arsel_mlp_train_step(context(self.device), ctypes.byref(self.c), _ptr(X),
                                        _ptr(alpha), B, lr, self.t, _ptr(self.loss),
                                        _stream(self.device))
        _check(rc, "arsel_mlp_train_step")
        return self.loss

    def forward(self, X: torch.Tensor, alpha: torch.Tensor, want_q: bool = False):
        """Q (int32 bit patterns of uint32) [R, M] and optionally q [R, M]."""
        R = X.shape[0]
        arsel._need(X, torch.int32, R * self.N, "X", self.device)
        arsel._need(alpha, torch.float32, R * self.M, "alpha", self.device)
        Q = torch.empty(R, self.M, dtype=torch.int32, device=self.device)
        q = torch.empty(R, self.M, dtype=torch.float32, device=self.device) if want_q else None
        rc = lib().arsel_mlp_forward(context(self.device), ctypes.byref(self.c.net), _ptr(X), R,
                                     _ptr(alpha), _ptr(q), _ptr(Q), _stream(self.device))
        _check(rc, "arsel_mlp_forward")
        return Q, q

    def state_dict(self) -> dict:
        return {"t": self.t, "master": [t.clone() for t in self.master],
                "m": [t.clone() for t in self.m], "v": [t.clone() for t in self.v]}

    def load_state_dict(self, sd: dict) -> None:
        self.t = int(sd["t"])
        for dst, src in zip(self.master + self.m + self.v, sd["master"] + sd["m"] + sd["v"]):
            dst.copy_(src)
        self.sync()
