"""Profiling helpers: counter calibration and rocprofv3 summaries.

    python -m paper_1404_0027_amd.profiling copy
        Runs a plain device copy of known size (64 MiB read, 64 MiB written,
        20 times) so that the FETCH_SIZE / WRITE_SIZE counters can be
        calibrated: factor = true KiB / counter KiB per dispatch.

    python -m paper_1404_0027_amd.profiling ragged [WAVE_MAX_M BLOCK_WAVES LDS_MAX_M BLOCKS_PER_CU]
        Runs the uneven-batch call 12 times on the benchmark's 10^4-instance
        batch (host-built work lists, indices only) with the given schedule
        (default 1024 8 0 4), for kernel traces and counters of its launches.

    python -m paper_1404_0027_amd.profiling dense
        Runs the dense selection 40 times on the benchmark's batch (R = 4096
        realizations x M = 1029, SoA, lognormal(0,2) with 30% zeros, 32
        rotating buffers; k_select_tile<16>) and 5 times on 10^6
        realizations of the same law (k_select_tile<8>), for counters of both
        launch shapes.

    python -m paper_1404_0027_amd.profiling ssa
        Runs the full SSA on the benchmark's network (N = 641, M = 1029, counts
        Poisson(50)), R = 16384 realizations x 2000 steps, once with envelopes
        maintained between exact steps every 64 (k_ssa_run_pair) and once
        exact at every step (k_ssa_run), for counters of both run kernels.

    python -m paper_1404_0027_amd.profiling summarize DB KERNEL_SUBSTR [--pmc]
        Prints per-kernel dispatch count and mean/min/max duration from a
        rocprofv3 kernel-trace database, or mean counter values per dispatch
        (--pmc), for kernels whose name contains KERNEL_SUBSTR.

    python -m paper_1404_0027_amd.profiling traffic FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB KERNEL OUT.json
        Scales the kernel's FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by
        the copy calibration and writes bytes per launch with a hash of the
        kernel sources, so the benchmark only reports traffic measured on the
        current kernels.
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_MIB = 64


# sources each profiled kernel is compiled from (its traffic record is void
# once any of them changes)
_RAGGED_SOURCES = ("select_ragged.hip", "select_block.hpp", "select_core.hpp", "wave_reduce.hpp",
                   "device.hpp", "launch.hpp")
KERNEL_SOURCES = {
    "select_tile": ("select_dense.hip", "select_core.hpp", "device.hpp", "launch.hpp"),
    "ragged_scan": _RAGGED_SOURCES,
    "ragged_hard": _RAGGED_SOURCES,
}


def source_hash(kernel: str = "select_tile") -> str:
    h = hashlib.sha256()
    names = KERNEL_SOURCES.get(kernel)
    paths = ([os.path.join(HERE, "csrc", n) for n in names] if names
             else sorted(glob.glob(os.path.join(HERE, "csrc", "*"))))
    for p in paths:
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def copy_probe() -> None:
    import torch

    n = COPY_MIB * 1024 * 1024 // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty(n, device="cuda")
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy probe: 20 x {COPY_MIB} MiB device-to-device copies done", flush=True)


def ragged_probe(sched=(1024, 8, 0, 4)) -> None:
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1404_0027_amd import arsel, workloads

    rb = workloads.ragged_mix(K=10000, seed=3)
    a = torch.from_numpy(rb.alpha).cuda()
    off = torch.from_numpy(rb.offsets).cuda()
    idx = torch.empty(rb.K, dtype=torch.int32, device="cuda")
    arsel.set_schedule(arsel.Schedule(*sched))
    for s in range(12):
        arsel.select_ragged(a, off, seed=1, step=s, host_offsets=rb.offsets, index=idx)
    torch.cuda.synchronize()
    print(f"ragged probe: 12 calls, K={rb.K}, {4 * int(rb.offsets[-1])} B of propensities, "
          f"schedule {tuple(sched)}", flush=True)


def dense_probe() -> None:
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1404_0027_amd import arsel, workloads

    M, R, nbuf = 1029, 4096, 32
    bufs = torch.from_numpy(workloads.lognormal_soa(M=M, K=R, seed=2, buffers=nbuf)).cuda()
    idx = torch.empty(R, dtype=torch.int32, device="cuda")
    for s in range(40):
        arsel.select(bufs[s % nbuf], M, R, R, arsel.SOA, seed=1, step=s, index=idx)
    torch.cuda.synchronize()
    del bufs
    K = 1_000_000
    g = torch.Generator(device="cuda").manual_seed(123)
    a = torch.empty(M, K, device="cuda")
    for r in range(0, M, 64):
        blk = a[r:r + 64]
        blk.log_normal_(0.0, 2.0, generator=g)
        blk[torch.rand(blk.shape, device="cuda", generator=g) < 0.3] = 0.0
    big = torch.empty(K, dtype=torch.int32, device="cuda")
    for s in range(5):
        arsel.select(a, M, K, K, arsel.SOA, seed=1, step=s, index=big)
    torch.cuda.synchronize()
    print(f"dense probe: 40 launches of {R} x {M}, 5 launches of {K} x {M}", flush=True)


def ssa_probe() -> None:
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1404_0027_amd import learned, workloads

    net = workloads.mass_action_network()
    dn = learned.DeviceNetwork(net)
    R, steps = 16384, 2000
    X0 = torch.from_numpy(workloads.poisson_counts(N=net.N, R=R, seed=5)).cuda()
    for period in (64, 1):
        X = X0.clone()
        t = torch.zeros(R, dtype=torch.float64, device="cuda")
        dn.run(X, t, seed=1, step0=0, steps=steps, period=period)
    torch.cuda.synchronize()
    print(f"ssa probe: {R} realizations x {steps} steps at periods 64 and 1", flush=True)


def _kernel_rows(db: str, substr: str):
    c = sqlite3.connect(db)
    return c.execute("select name, start, end from kernels where name like ?",
                     (f"%{substr}%",)).fetchall()


def _pmc_rows(db: str, substr: str):
    c = sqlite3.connect(db)
    return c.execute("select kernel_name, counter_name, avg(value), count(*) from counters_collection "
                     "where kernel_name like ? group by kernel_name, counter_name",
                     (f"%{substr}%",)).fetchall()


def summarize(db: str, substr: str, pmc: bool = False) -> str:
    lines = []
    if pmc:
        for name, counter, avg, n in _pmc_rows(db, substr):
            lines.append(f"{name[:70]:70s} {counter:16s} mean {avg:14.1f} per dispatch (n={n})")
        return "\n".join(lines)
    rows = _kernel_rows(db, substr)
    by = {}
    for name, s, e in rows:
        by.setdefault(name, []).append((e - s) / 1e3)
    for name, d in sorted(by.items()):
        d.sort()
        lines.append(f"{name[:70]:70s} n={len(d):6d} mean {sum(d)/len(d):9.3f} us  "
                     f"median {d[len(d)//2]:9.3f} us  min {d[0]:9.3f}  max {d[-1]:9.3f}")
    return "\n".join(lines)


def _counter(db: str, substr: str, counter: str) -> float:
    vals = [avg for name, c, avg, n in _pmc_rows(db, substr) if c == counter]
    if not vals:
        raise SystemExit(f"no {counter} for '{substr}' in {db}")
    return vals[0]


def traffic(fetch_db, write_db, copy_fetch_db, copy_write_db, kernel, out_json) -> dict:
    true_kib = COPY_MIB * 1024.0
    f_factor = true_kib / _counter(copy_fetch_db, "copy", "FETCH_SIZE")
    w_factor = true_kib / _counter(copy_write_db, "copy", "WRITE_SIZE")
    fetch = _counter(fetch_db, kernel, "FETCH_SIZE") * f_factor * 1024.0
    write = _counter(write_db, kernel, "WRITE_SIZE") * w_factor * 1024.0
    rec = {"kernel": kernel, "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write, "fetch_calibration": f_factor,
           "write_calibration": w_factor, "source_hash": source_hash(kernel)}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def main(argv: list[str]) -> int:
    if not argv:
        print(__doc__)
        return 2
    if argv[0] == "copy":
        copy_probe()
    elif argv[0] == "dense":
        dense_probe()
    elif argv[0] == "ssa":
        ssa_probe()
    elif argv[0] == "ragged":
        ragged_probe(tuple(int(x) for x in argv[1:5]) if len(argv) >= 5 else (1024, 8, 0, 4))
    elif argv[0] == "summarize":
        print(summarize(argv[1], argv[2], pmc="--pmc" in argv))
    elif argv[0] == "traffic":
        print(json.dumps(traffic(*argv[1:7])))
    elif argv[0] == "hash":
        print(source_hash(*argv[1:2]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
