"""Schedule autotuner for the selection kernels.

The schedule of a launch -- the size up to which an instance is staged in one
wavefront's LDS slice, waves per pick workgroup, the LDS piece (and chunk) of
the hard rows, pick workgroups per CU (uneven batches); instances per tile and
waves per workgroup (dense path) --
never changes results (every schedule returns the sequential rule's answer),
only speed.  The tuner times each candidate on the caller's own batch with
HIP events and keeps the fastest; choices are cached per device and workload
signature so a steady-state loop pays for the search once.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import arsel

CACHE_PATH = os.environ.get("ARSEL_AUTOTUNE_CACHE",
                            os.path.join(os.path.expanduser("~"), ".cache", "arsel_autotune.json"))


def ragged_candidates(lds_bytes: int) -> list[tuple[int, int, int, int]]:
    """(wave_max_m, block_waves, lds_max_m, blocks_per_cu) that fit the device."""
    out = []
    for wave_max_m in (256, 512, 1024, 2048, 4096):
        for block_waves in (4, 8, 16):
            for lds_max_m in (0, 4096, 8192):          # hard piece: 16380, 4096, 8192 floats
                for bpc in (1, 2, 4, 6, 8):
                    need = block_waves * wave_max_m * 4 + 2048
                    if need > lds_bytes or need * bpc > 160 * 1024:
                        continue
                    out.append((wave_max_m, block_waves, lds_max_m, bpc))
    return out


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps   # microseconds


def _signature(sizes: np.ndarray) -> str:
    """Workload key: K and a log2 histogram of the instance sizes."""
    hist = np.bincount(np.log2(np.maximum(sizes, 1)).astype(np.int64), minlength=32)[:32]
    return f"K{sizes.shape[0]}-" + "-".join(str(int(h)) for h in hist)


def _load_cache() -> dict:
    try:
        with open(CACHE_PATH) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE_PATH), exist_ok=True)
        tmp = CACHE_PATH + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1)
        os.replace(tmp, CACHE_PATH)
    except OSError:
        pass


@dataclass
class TuneResult:
    schedule: tuple
    micros: float
    table: list   # (schedule, microseconds) of every candidate tried


def tune_ragged(alpha: torch.Tensor, offsets: torch.Tensor, host_offsets: np.ndarray, *,
                candidates=None, reps: int = 3, use_cache: bool = True, seed: int = 1,
                device=None) -> TuneResult:
    """Pick the fastest ragged schedule for this batch and install it."""
    dev = alpha.device
    name = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    sizes = np.diff(np.asarray(host_offsets, dtype=np.int64))
    key = f"ragged/{name}/{_signature(sizes)}"
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache:
        sched = tuple(cache[key]["schedule"])
        arsel.set_schedule(arsel.Schedule(*sched), device=dev)
        return TuneResult(sched, cache[key]["micros"], [])
    lds_bytes = torch.cuda.get_device_properties(dev).shared_memory_per_block
    cands = candidates or ragged_candidates(lds_bytes)
    index = torch.empty(sizes.shape[0], dtype=torch.int32, device=dev)
    table = []
    for c in cands:
        try:
            arsel.set_schedule(arsel.Schedule(*c), device=dev)
        except arsel.ArselError:
            continue
        us = _time(lambda: arsel.select_ragged(alpha, offsets, seed=seed, step=0,
                                               host_offsets=host_offsets, index=index), reps)
        table.append((c, us))
    best = min(table, key=lambda x: x[1])
    arsel.set_schedule(arsel.Schedule(*best[0]), device=dev)
    if use_cache:
        cache[key] = {"schedule": list(best[0]), "micros": best[1]}
        _save_cache(cache)
    return TuneResult(best[0], best[1], table)


def tune_dense(alpha: torch.Tensor, M: int, K: int, ld: int, layout: int, *, reps: int = 20,
               candidates=((16, 16), (8, 8), (16, 8), (32, 16), (8, 4), (4, 4)),
               seed: int = 1) -> TuneResult:
    """Pick the fastest dense (tile, waves) for this shape and install it."""
    dev = alpha.device
    index = torch.empty(K, dtype=torch.int32, device=dev)
    table = []
    for tile, waves in candidates:
        arsel.set_dense_config(tile, waves, device=dev)
        us = _time(lambda: arsel.select(alpha, M, K, ld, layout, seed=seed, index=index), reps)
        table.append(((tile, waves), us))
    best = min(table, key=lambda x: x[1])
    arsel.set_dense_config(*best[0], device=dev)
    return TuneResult(best[0], best[1], table)
