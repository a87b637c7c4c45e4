"""Benchmark: batched acceptance-rejection next-reaction selection on one MI355X.

Workload: R = 4096 realizations, each with its own FP32 propensity vector of
M = 1029 reactions (lognormal(0,2), 30% set exactly to zero), stored SoA
(alpha[j*4096 + k]); one selection per realization per step; 32 distinct
propensity batches (540 MB, more than the 256 MB Infinity Cache) rotated
across steps; Philox4x32-10 seed 1, step counter = step index.  The K timed
steps are captured in one HIP graph and replayed once between HIP events.

Prints one JSON line: selections/s, the roofline of the selection kernel
(algorithmic bytes: 4 B per propensity + 4 B per index), the per-trial
acceptance of uniform AR on this workload, and the CPU oracle timed on a
bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M, R, NBUF, SEED = 1029, 4096, 32, 1
BYTES_PER_SELECTION = 4 * M + 4
HBM_PEAK_GBS = 8000.0


def load_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    from paper_1404_0027_amd.profiling import source_hash

    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash(kernel):
        return None
    return rec.get("bytes_per_launch")


def host_identity() -> dict:
    """Host CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def cpu_baseline(buf_host, threads: int, last_step: int, gpu_index, budget_s: float = 8.0):
    """The oracle timed on the host cores on a bounded sample of the same
    workload, once on `threads` cores (OpenMP over instances) and once on one
    core; it also recomputes the last timed GPU step for a parity check."""
    import numpy as np
    import oracle

    ref = oracle.select_uniform(buf_host[last_step % NBUF], M, R, R, oracle.SOA, seed=SEED,
                                step=last_step, threads=threads, want_alpha0=False,
                                want_trials=False)[0]
    parity = ("ok" if np.array_equal(gpu_index, ref)
              else f"MISMATCH ({int((gpu_index != ref).sum())} of {R})")

    def leg(nthreads: int, budget: float):
        t0 = time.perf_counter()
        oracle.select_uniform(buf_host[0], M, R, R, oracle.SOA, seed=SEED, step=0,
                              threads=nthreads, want_alpha0=False, want_trials=False)
        one = time.perf_counter() - t0
        steps = max(1, min(NBUF * 8, int(budget / max(one, 1e-6))))
        t0 = time.perf_counter()
        for s in range(steps):
            oracle.select_uniform(buf_host[s % NBUF], M, R, R, oracle.SOA, seed=SEED, step=s,
                                  threads=nthreads, want_alpha0=False, want_trials=False)
        return steps, time.perf_counter() - t0

    steps, dt = leg(threads, budget_s)
    steps1, dt1 = leg(1, budget_s)
    host = host_identity()
    return ({"value": steps * R / dt, "unit": "selections/s", "cores": threads, "kind": "oracle",
             "sample": f"{steps} steps x {R} realizations of the same workload (M={M} SoA), "
                       f"sequential AR per instance, OpenMP over instances on {threads} threads",
             "single_core": {"value": steps1 * R / dt1, "unit": "selections/s", "cores": 1,
                             "sample": f"{steps1} steps x {R} realizations, one thread"},
             "host": host}, parity)


def bench_ragged(torch, arsel, workloads, reps: int = 20):
    """Uneven batch: 10^4 instances, M log-uniform in [64, 65536], with the
    autotuned schedule: four launches per call (scan, split, hard chunks,
    pick).  Also timed: the same call with the work lists built on the device
    (what a captured call does) and the no-allocation entry point."""
    from paper_1404_0027_amd import autotune

    rb = workloads.ragged_mix(K=10000, seed=3)
    a = torch.from_numpy(rb.alpha).cuda()
    off = torch.from_numpy(rb.offsets).cuda()
    tuned = autotune.tune_ragged(a, off, rb.offsets, reps=5, use_cache=False)
    index = torch.empty(rb.K, dtype=torch.int32, device="cuda")
    calls = {
        "host_lists": lambda s: arsel.select_ragged(a, off, seed=SEED, step=s, host_offsets=rb.offsets,
                                                   index=index),
        "device_lists": lambda s: arsel.select_ragged(a, off, seed=SEED, step=s, index=index),
        "noalloc": lambda s: arsel.select_ragged_noalloc(a, off, seed=SEED, step=s, index=index),
    }
    us = {}
    for name, fn in calls.items():
        for s in range(3):
            fn(s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for s in range(reps):
            fn(s)
        e1.record()
        torch.cuda.synchronize()
        us[name] = e0.elapsed_time(e1) * 1e3 / reps
    t = us["host_lists"]
    nbytes = 4 * int(rb.offsets[-1]) + 4 * rb.K
    return {"workload": "10^4 instances, M = round(2^U(6,16)), families U(0,1]/Exp(1)/LN(0,3), "
                        "ragged AoS, host-built work lists reused across calls",
            "instances_per_s": round(rb.K / (t * 1e-6), 1), "us_per_launch": round(t, 2),
            "algorithmic_bytes": nbytes, "achieved_GBs": round(nbytes / (t * 1e-6) / 1e9, 1),
            "frac_of_8TBs": round(nbytes / (t * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "us_device_lists": round(us["device_lists"], 2), "us_noalloc": round(us["noalloc"], 2),
            "traffic_bytes_per_launch": {"k_ragged_scan": load_traffic("ragged_scan"),
                                         "k_ragged_hard": load_traffic("ragged_hard")},
            "schedule": dict(zip(("wave_max_m", "block_waves", "lds_max_m", "blocks_per_cu"),
                                 tuned.schedule)),
            "tuner_reps": 5}


def law_pvalue_rows(np, alpha_rows, rows, sel, bins: int = 64, seed: int = 0):
    """p-value that selections `sel` (index chosen for row rows[i] of
    alpha_rows [R, M]) follow alpha_j / alpha_0 of their own rows: the
    randomised probability integral transform F(j-) + V p_j is U(0,1) under
    that law; chi-square of its histogram over `bins` equal cells."""
    from scipy.stats import chi2

    a = np.asarray(alpha_rows, np.float64)
    P = a / a.sum(axis=1, keepdims=True)
    C = np.cumsum(P, axis=1)
    rows = np.asarray(rows)
    sel = np.asarray(sel, np.int64)
    if np.any(sel < 0):
        return 0.0
    hi = C[rows, sel]
    lo = hi - P[rows, sel]
    u = lo + np.random.default_rng(seed).random(sel.size) * (hi - lo)
    h = np.bincount(np.minimum((u * bins).astype(np.int64), bins - 1), minlength=bins)
    e = sel.size / bins
    return float(chi2.sf(((h - e) ** 2 / e).sum(), bins - 1))


def law_pvalue_counts(np, alpha, counts):
    """Chi-square p-value of selection counts of one vector against
    alpha_j / alpha_0 (cells with expectation below 5 merged)."""
    from scipy.stats import chi2

    p = np.asarray(alpha, np.float64)
    p = p / p.sum()
    c = np.asarray(counts, np.float64)
    n = c.sum()
    e = n * p
    keep = e >= 5
    obs = list(c[keep])
    exp = list(e[keep])
    if (~keep).any():
        obs.append(c[~keep].sum())
        exp.append(e[~keep].sum())
    obs, exp = np.asarray(obs), np.asarray(exp)
    return float(chi2.sf(((obs - exp) ** 2 / exp).sum(), obs.size - 1))


def _acceptance(np, trials):
    t = trials.cpu().numpy().view(np.uint32).astype(np.int64)
    ok = (t >= 1) & (t <= 4096)
    return float(ok.sum() / max(1, t[ok].sum() + 4096 * (t > 4096).sum()))


def _timed(torch, fn, reps):
    """Seconds per call of fn(step): `reps` calls captured in one HIP graph,
    replayed between events (so host-side call overhead is not timed)."""
    fn(0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap, capture_error_mode="relaxed"):
            for s in range(reps):
                fn(s + 1)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def bench_learned(torch, np, arsel, workloads, epochs: int = 8, lr0: float = 2e-3,
                  decay: float = 0.5):
    """Learned proposal on the synthetic mass-action network (N=641, M=1029):
    10^6 (state, propensity) pairs from GPU jump chains, training on the GPU,
    then acceptance and selections/s against uniform AR on held-out states
    drawn from the same chains' distribution (fresh seeds)."""
    from paper_1404_0027_amd import learned

    net = workloads.mass_action_network()
    dn = learned.DeviceNetwork(net)
    X0 = torch.from_numpy(workloads.poisson_counts(N=net.N, R=1000, seed=5)).cuda()
    dn.chain(X0, seed=2, step0=0, steps=1000)
    rec, _ = dn.chain(X0, seed=2, step0=1000, steps=1000, record_from=0)
    X = rec.reshape(-1, net.N)
    alpha = dn.propensities(X)
    lp = learned.LearnedProposal(net.N, net.M, seed=0)
    B = 1024
    n = (X.shape[0] // B) * B
    order = torch.randperm(n // B, generator=torch.Generator().manual_seed(0)).tolist()
    t0 = time.perf_counter()
    for e in range(epochs):
        lr = lr0 * decay ** e
        for b in order:
            lp.train_step(X[b * B:(b + 1) * B], alpha[b * B:(b + 1) * B], lr=lr)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    loss = float(lp.loss.item())
    del rec, X, alpha
    # held-out: 4096 fresh realizations, 1500 steps (inside the training window)
    Xh = torch.from_numpy(workloads.poisson_counts(N=net.N, R=4096, seed=77)).cuda()
    dn.chain(Xh, seed=9, step0=0, steps=1500)
    Ah = dn.propensities(Xh)
    Q, _ = lp.forward(Xh, Ah)
    Rh = Xh.shape[0]
    idx = torch.empty(Rh, dtype=torch.int32, device="cuda")
    tr = torch.empty(Rh, dtype=torch.int32, device="cuda")

    # (a) one selection per distinct state: alpha and Q read once per selection
    arsel.select(Ah, net.M, Rh, net.M, arsel.AOS, seed=SEED, index=idx, trials=tr)
    acc_u = _acceptance(np, tr)
    arsel.select_proposal(Ah, Q, seed=SEED, index=idx, trials=tr)
    acc_l = _acceptance(np, tr)
    t_u = _timed(torch, lambda s: arsel.select(Ah, net.M, Rh, net.M, arsel.AOS, seed=SEED, step=s,
                                               index=idx), 200)
    t_p = _timed(torch, lambda s: arsel.select_proposal(Ah, Q, seed=SEED, step=s, index=idx), 200)

    def full(s):
        lp.forward(Xh, Ah)
        arsel.select_proposal(Ah, Q, seed=SEED, step=s, index=idx)

    t_f = _timed(torch, full, 50)

    # selection law of the timed launches: 20 steps of each path, every
    # selection against its own state's alpha_j / alpha_0
    Ah_np = Ah.cpu().numpy()
    law = {}
    for name, call in (("uniform_AR", lambda s: arsel.select(Ah, net.M, Rh, net.M, arsel.AOS,
                                                             seed=SEED, step=s, index=idx)),
                       ("learned", lambda s: arsel.select_proposal(Ah, Q, seed=SEED, step=s,
                                                                   index=idx))):
        sel = []
        for s in range(1, 21):
            call(s)
            sel.append(idx.cpu().numpy().copy())
        sel = np.concatenate(sel)
        law[name] = round(law_pvalue_rows(np, Ah_np, np.tile(np.arange(Rh), 20), sel), 4)

    # (b) ensembles from common states: K selections from each of 8 held-out
    # states (the first step of K realizations started from that state)
    K = 1 << 20
    bi = torch.empty(K, dtype=torch.int32, device="cuda")
    bt = torch.empty(K, dtype=torch.int32, device="cuda")
    rates_u, rates_l, accs_u, accs_l, ens_p = [], [], [], [], []
    for s in range(8):
        a1, q1 = Ah[s].contiguous(), Q[s].contiguous()
        arsel.select(a1, net.M, K, 0, arsel.AOS, seed=SEED, index=bi, trials=bt)
        accs_u.append(_acceptance(np, bt))
        arsel.select_proposal_broadcast(a1, q1, K, seed=SEED, index=bi, trials=bt)
        accs_l.append(_acceptance(np, bt))
        rates_u.append(K / _timed(torch, lambda st: arsel.select(a1, net.M, K, 0, arsel.AOS,
                                                                  seed=SEED, step=st, index=bi), 20))
        rates_l.append(K / _timed(torch, lambda st: arsel.select_proposal_broadcast(
            a1, q1, K, seed=SEED, step=st, index=bi), 20))
        # the last timed launch's K selections against this state's law
        cnt = torch.bincount(bi.long(), minlength=net.M)[:net.M].cpu().numpy()
        ens_p.append(law_pvalue_counts(np, a1.cpu().numpy(), cnt))
    ru, rl = float(np.mean(rates_u)), float(np.mean(rates_l))
    return {"workload": "mass-action network N=641, M=1029, counts Poisson(50); MLP "
                        "641->256->256->1029 BF16 on MFMA; held-out states = 4096 fresh "
                        "realizations after 1500 jump-chain steps",
            "training": {"pairs": int(n), "epochs": epochs, "batch": B, "lr": [lr0, decay],
                         "order": "minibatches shuffled once (seed 0), Adam",
                         "seconds": round(train_s, 2), "final_minibatch_loss": round(loss, 4)},
            "per_state": {
                "what": "4096 distinct states, one selection each (alpha and Q read once per "
                        "selection: HBM-bound, the proposal doubles the bytes)",
                "acceptance_per_trial": {"uniform": round(acc_u, 5), "learned": round(acc_l, 5),
                                         "gain": round(acc_l / acc_u, 2)},
                "selections_per_s": {"uniform_AR": round(Rh / t_u, 1),
                                     "learned_select_only": round(Rh / t_p, 1),
                                     "learned_with_MLP_forward": round(Rh / t_f, 1)},
                "law_chi2_p": dict(law, what="20 launches x 4096 selections per path, each "
                                   "against its own state's alpha_j / alpha_0 (randomised "
                                   "PIT, 64 cells)")},
            "ensemble": {
                "what": f"{K} selections from each of 8 held-out states (alpha, Q staged once; "
                        "trial-bound), automatic trial width for both",
                "acceptance_per_trial": {"uniform": round(float(np.mean(accs_u)), 5),
                                         "learned": round(float(np.mean(accs_l)), 5)},
                "selections_per_s": {"uniform_AR": round(ru, 1), "learned": round(rl, 1),
                                     "speedup": round(rl / ru, 2)},
                "learned_law_chi2_p": {"per_state": [round(x, 4) for x in ens_p],
                                       "what": "the last timed learned launch (2^20 selections) "
                                               "of each state against alpha_j / alpha_0"}}}, lp


def bench_ssa(torch, np, arsel, workloads, lp=None, refresh: int = 1000, period: int = 64):
    """Full batched SSA on the N=641 / M=1029 mass-action network: R = 16384
    realizations x 10^4 steps, one launch (selection, time step,
    stoichiometry, dependency-graph propensity updates per step), with the
    envelopes exact at every step (period 1) and maintained from the changed
    propensities (exact every `period` steps).  With a trained proposal
    network lp, also the same runs selecting with its proposal, refreshed
    every `refresh` steps (MLP forward on the current states, inside the
    timed region)."""
    from paper_1404_0027_amd import learned

    net = workloads.mass_action_network()
    dn = learned.DeviceNetwork(net)
    R, steps = 16384, 10000
    X0 = torch.from_numpy(workloads.poisson_counts(N=net.N, R=R, seed=5)).cuda()
    X = X0.clone()
    t = torch.zeros(R, dtype=torch.float64, device="cuda")
    dn.run(X, t, seed=SEED, step0=0, steps=100)            # warm-up (and the dependency graph)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        X.copy_(X0)
        t.zero_()
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3

    sec = {p: timed(lambda: dn.run(X, t, seed=SEED, step0=0, steps=steps, period=p))
           for p in (1, period)}
    sim_t = float(t.mean().item())
    # the jump chain kernel (full propensity recompute each step) for reference
    X.copy_(X0)
    torch.cuda.synchronize()
    e0.record()
    dn.chain(X, seed=SEED, step0=0, steps=1000)
    e1.record()
    torch.cuda.synchronize()
    sec_chain = e0.elapsed_time(e1) * 1e-3 * (steps / 1000)
    out = {"workload": "full SSA, mass-action network N=641, M=1029, counts Poisson(50): "
                       f"R={R} realizations x {steps} steps in one launch",
           "selections_per_s": round(R * steps / sec[period], 1),
           "seconds": round(sec[period], 4), "period": period,
           "exact_envelope_every_step": {"selections_per_s": round(R * steps / sec[1], 1),
                                         "seconds": round(sec[1], 4)},
           "mean_simulated_time": sim_t,
           "jump_chain_full_recompute_selections_per_s": round(R * steps / sec_chain, 1),
           "note": "per step: AR selection against the step's envelope, tau, stoichiometry, "
                   "propensities of the affected reactions; envelopes exact every "
                   f"{period} steps (one pass over the LDS-resident propensities), kept from "
                   "the changed propensities between; alpha_0 of tau exact at every step "
                   "(128-bit fixed-point sum kept from the changes, rounded once), so the "
                   "times are bit-identical to the sequential definition"}
    if lp is None:
        return out

    # the network's Q sums to about 2^(31 - ceil(log2 M)); reactions it left
    # out (inactive at the refresh) weigh about 1/8 of an average one
    qfloor = (1 << (31 - (net.M - 1).bit_length())) // (8 * net.M)

    def learned_run(p, acc=None):
        for seg in range(0, steps, refresh):
            a = dn.propensities(X)
            Q, _ = lp.forward(X, a)
            if acc is not None:       # acceptance per trial on the refresh states
                tr = torch.empty(R, dtype=torch.int32, device="cuda")
                arsel.select(a, net.M, R, net.M, arsel.AOS, seed=SEED, step=seg, trials=tr)
                acc["uniform"].append(_acceptance(np, tr))
                arsel.select_proposal(a, Q, seed=SEED, step=seg, trials=tr)
                acc["learned"].append(_acceptance(np, tr))
            fired, _ = dn.run(X, t, seed=SEED, step0=seg, steps=min(refresh, steps - seg), Q=Q,
                              qfloor=qfloor, period=p, want_fired=acc is not None)
            if acc is not None:       # the segment's first step selected from the refresh states
                acc["law_a"].append(a.cpu().numpy())
                acc["law_sel"].append(fired[0].cpu().numpy())

    acc = {"uniform": [], "learned": [], "law_a": [], "law_sel": []}
    timed(lambda: learned_run(period, acc))                 # (acceptance pass)
    sec_l = {p: timed(lambda: learned_run(p)) for p in (1, period)}
    out["with_learned_proposal"] = {
        "what": f"same runs, steps select with the trained network's proposal "
                f"Q' = max(Q, {qfloor}), Q refreshed every {refresh} steps (MLP forward timed)",
        "selections_per_s": round(R * steps / sec_l[period], 1),
        "seconds": round(sec_l[period], 4),
        "exact_envelope_every_step_selections_per_s": round(R * steps / sec_l[1], 1),
        "speedup_vs_uniform": round(sec[period] / sec_l[period], 3),
        "acceptance_per_trial_at_refresh": {
            "uniform": round(float(np.mean(acc["uniform"])), 5),
            "learned": round(float(np.mean(acc["learned"])), 5)},
        "law_chi2_p_first_steps": round(law_pvalue_rows(
            np, np.concatenate(acc["law_a"]), np.arange(R * len(acc["law_a"])),
            np.concatenate(acc["law_sel"])), 4),
        "law_what": "the first step of each refresh segment (16384 realizations x "
                    f"{steps // refresh} segments) against its state's alpha_j / alpha_0 "
                    "(randomised PIT, 64 cells); the acceptance pass is a separate, untimed run",
        "mean_simulated_time": float(t.mean().item())}
    return out


K_GRID = (100, 1000, 10000, 50000, 62500)      # the paper's K values (Table 1, Fig. 2)
N_TABLE1 = 10_000_000                             # selections per Table 1 cell


def _counts_of(torch, fn, K: int, n: int, M: int):
    """Run ceil(n / K) launches of fn(step, index_view) writing consecutive
    slices of one index buffer; returns the counts of 0..M-1 and of -5."""
    launches = (n + K - 1) // K
    allidx = torch.empty(launches * K, dtype=torch.int32, device="cuda")
    for s in range(launches):
        fn(s, allidx[s * K:(s + 1) * K])
    sel = allidx[:n]
    rej = int((sel == -5).sum().item())
    counts = torch.bincount(sel.clamp(min=0).long(), minlength=M)[:M]
    counts[0] -= int((sel < 0).sum().item())          # the clamped statuses
    return counts.cpu().numpy(), rej


def bench_paper_table1(torch, np, arsel, workloads):
    """The paper's Table 1 grid: 10^7 selections from each discrete Gaussian
    (M = 64, 256, 1024) for every K in the paper's grid and both thresholds
    T_w = w * alpha_max (w = 1, 2), the paper's election/selection scheme
    against exact AR: MSE between alpha / alpha_0 and the observed
    frequencies (over accepted selections), rejections (failed elections)
    against the closed-form law's expectation, and selections/s of each
    (graph replays of 20 launches)."""
    gold_path = os.path.join(ROOT, "tests", "golden", "paper_scheme_expectations.json")
    with open(gold_path) as f:
        gold = json.load(f)["rows"]
    out = {}
    for M in (64, 256, 1024):
        a_np = workloads.gaussian_vector(M)
        a = torch.from_numpy(a_np).cuda()
        p = a_np.astype(np.float64) / a_np.astype(np.float64).sum()
        rows = {}
        for K in K_GRID:
            cell = {}
            for w in (1, 2):
                fn = (lambda s, ix, w=w, K=K: arsel.select_paper(a, M, K, 0, w=float(w), seed=SEED,
                                                                  step=s, index=ix))
                c, rej = _counts_of(torch, fn, K, N_TABLE1, M)
                freq = c / max(1, c.sum())
                ix = torch.empty(K, dtype=torch.int32, device="cuda")
                g = gold[str(M)][f"T{w}"]
                cell[f"paper_T{w}"] = {
                    "mse": float(np.mean((freq - p) ** 2)), "law_mse": g["expected_mse"],
                    "rejections": rej, "law_rejections": round(g["expected_rejections"], 3),
                    "selections_per_s": round(K / _timed(torch, lambda s: fn(s, ix), 20), 1)}
            fx = (lambda s, ix, K=K: arsel.select(a, M, K, 0, arsel.AOS, seed=SEED, step=s,
                                                  index=ix))
            c, rej = _counts_of(torch, fx, K, N_TABLE1, M)
            ix = torch.empty(K, dtype=torch.int32, device="cuda")
            cell["exact_AR"] = {"mse": float(np.mean((c / c.sum() - p) ** 2)),
                                "sampling_floor_mse": gold[str(M)]["exact_sampling_floor_mse"],
                                "statuses_below_zero": rej,
                                "selections_per_s": round(K / _timed(torch, lambda s: fx(s, ix), 20), 1)}
            rows[str(K)] = cell
        out[str(M)] = rows
    return {"workload": "discrete Gaussian propensities (section on test and validation), "
                        f"{N_TABLE1} selections per cell, K in {list(K_GRID)}, "
                        "T_w = w * alpha_max for the paper's scheme",
            "by_M_then_K": out,
            "note": "MSE = mean_j (alpha_j / alpha_0 - observed frequency_j)^2 over accepted "
                    "selections; each cell is ONE run (the paper prints the worst of 10); law_* "
                    "are the closed-form law's expectations (tests/golden/"
                    "paper_scheme_expectations.json, written by the oracle); exact AR sits at the "
                    "multinomial sampling floor, the paper's scheme adds its bias"}


def bench_k_sweep(torch, np, arsel, workloads):
    """Selections/s against K for M = 64, 256, 1024 (the shape of the paper's
    timing study, section "Performance and scalability of the algorithm"):
    exact uniform AR, (a) one shared discrete Gaussian vector broadcast to K
    instances (the paper's setting), (b) K distinct lognormal(0,2) vectors with
    30% zeros, SoA, rotated over enough buffers to exceed the 256 MB Infinity
    Cache where K * M allows (at most 32).  Graph replays of 50 launches."""
    out = {}
    for M in (64, 256, 1024):
        g = torch.from_numpy(workloads.gaussian_vector(M)).cuda()
        rows = {}
        for K in K_GRID:
            ix = torch.empty(K, dtype=torch.int32, device="cuda")
            t_sh = _timed(torch, lambda s: arsel.select(g, M, K, 0, arsel.AOS, seed=SEED, step=s,
                                                        index=ix), 50)
            nb = int(min(32, max(1, -(-600_000_000 // (4 * M * K)))))
            bufs = [_scale_input(torch, M, K, 1000 + b) for b in range(nb)]
            t_d = _timed(torch, lambda s: arsel.select(bufs[s % nb], M, K, K, arsel.SOA, seed=SEED,
                                                       step=s, index=ix), 50)
            nbytes = K * (4 * M + 4)
            rows[str(K)] = {
                "shared_vector": {"selections_per_s": round(K / t_sh, 1),
                                  "ms_per_1e7_selections": round(1e10 * t_sh / K, 3)},
                "distinct_vectors": {"selections_per_s": round(K / t_d, 1),
                                     "ms_per_1e7_selections": round(1e10 * t_d / K, 3),
                                     "us_per_launch": round(t_d * 1e6, 3),
                                     "achieved_GBs": round(nbytes / t_d / 1e9, 1),
                                     "buffers": nb}}
            del bufs
        out[str(M)] = rows
    torch.cuda.empty_cache()
    return {"workload": "exact uniform AR, K instances x M reactions per launch; shared = one "
                        "discrete Gaussian vector for all instances (broadcast), distinct = SoA "
                        "lognormal(0,2) with 30% zeros per instance",
            "by_M_then_K": out,
            "paper_reference": "GPU/AR: 2277.18 ms on a Tesla M2075 and 1326.78 ms on a K20 for "
                               "10^7 selections at M = 1024, K = 62500 (section 'Performance and "
                               "scalability of the algorithm'; other hardware, context only)"}


def _scale_input(torch, M: int, K: int, seed: int):
    """SoA [M][K] lognormal(0,2) with 30% exact zeros, generated on the GPU in
    row chunks (no [M][K] temporary)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    a = torch.empty(M, K, device="cuda")
    for r in range(0, M, 64):
        blk = a[r:r + 64]
        blk.log_normal_(0.0, 2.0, generator=g)
        blk[torch.rand(blk.shape, device="cuda", generator=g) < 0.3] = 0.0
    return a


def bench_ceiling(torch, arsel, bufs, reps: int = 200):
    """Achievable read bandwidth (arsel_probe_read) on the headline batch
    shape and at 10^6 realizations: the same bytes read once with the
    selection kernels' loads and nothing else, as graph replays over the same
    rotating buffers (per-launch time includes the graph's launch gap)."""
    nb, Mb, Rb = bufs.shape
    out = {}
    for tile in (0, 16):
        sink = arsel.probe_read(bufs[0], Mb, Rb, Rb, tile)
        sec = _timed(torch, lambda s: arsel.probe_read(bufs[s % nb], Mb, Rb, Rb, tile, sink=sink),
                     reps)
        nbytes = 4 * Mb * Rb
        out["contiguous" if tile == 0 else f"soa_tile{tile}"] = {
            "us_per_launch": round(sec * 1e6, 3), "GBs": round(nbytes / sec / 1e9, 1)}
    big = _scale_input(torch, 1029, 1_000_000, 321)
    for tile in (0, 16):
        sink = arsel.probe_read(big, 1029, 1_000_000, 1_000_000, tile)
        sec = _timed(torch, lambda s: arsel.probe_read(big, 1029, 1_000_000, 1_000_000, tile,
                                                       sink=sink), 10)
        out[("contiguous" if tile == 0 else f"soa_tile{tile}") + "_1e6x1029"] = {
            "us_per_launch": round(sec * 1e6, 1), "GBs": round(4 * 1029e6 / sec / 1e9, 1)}
    del big
    # an empty launch: the probe on zero rows (one graph node, no work)
    sink = arsel.probe_read(bufs[0], 0, 16, 16, 0)
    out["empty_launch_us"] = round(_timed(torch, lambda s: arsel.probe_read(
        bufs[0], 1, 16, 16, 0, sink=sink), reps) * 1e6, 3)
    torch.cuda.empty_cache()
    return out


def bench_scale(torch, K: int = 1_000_000, reps: int = 10):
    """The dense kernel at the paper's scale claims: K realizations x M = 1029
    (SoA, lognormal(0,2) with 30% zeros) in one launch -- 10^6 (4.1 GB), and
    the sensitivity-analysis shape 9 x 1029 x 1000 = 9,261,000 (38 GB)."""
    from paper_1404_0027_amd import arsel

    Mb = 1029
    a = _scale_input(torch, Mb, K, 123)
    idx = torch.empty(K, dtype=torch.int32, device="cuda")
    sec = _timed(torch, lambda s: arsel.select(a, Mb, K, K, arsel.SOA, seed=SEED, step=s,
                                                index=idx), reps)
    nbytes = K * (4 * Mb + 4)
    del a
    torch.cuda.empty_cache()
    return {"workload": f"{K} realizations x M={Mb} SoA (lognormal(0,2), 30% zeros), one launch",
            "selections_per_s": round(K / sec, 1), "us_per_launch": round(sec * 1e6, 1),
            "algorithmic_bytes": nbytes, "achieved_GBs": round(nbytes / sec / 1e9, 1),
            "frac_of_8TBs": round(nbytes / sec / 1e9 / HBM_PEAK_GBS, 4)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tile", type=int, default=0, help="dense tile override (results unchanged)")
    ap.add_argument("--waves", type=int, default=0, help="dense waves override (results unchanged)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the uneven-batch and learned-proposal measurements")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(instances are independent: the multi-GPU design shards realizations, "
              f"see the design notes)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1404_0027_amd import arsel, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] generating {NBUF} x {M} x {R} propensities", file=sys.stderr, flush=True)
    host = workloads.lognormal_soa(M=M, K=R, seed=2, buffers=NBUF)
    bufs = torch.from_numpy(host).to(dev)
    index = torch.empty(R, dtype=torch.int32, device=dev)
    arsel.context(0)
    if args.tile or args.waves:
        arsel.set_dense_config(args.tile or 16, args.waves or 16)

    def launch(s: int):
        b = bufs[s % NBUF]
        arsel.select(b, M, R, R, arsel.SOA, seed=SEED, step=s, index=index)

    for s in range(args.warmup):
        launch(s)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} steps done; capturing {args.steps}", file=sys.stderr,
          flush=True)

    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap, capture_error_mode="relaxed"):
            for s in range(args.steps):
                launch(s)
    torch.cuda.synchronize()

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    g.replay()
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    sel_per_s = args.steps * R / (ms * 1e-3)
    avg_launch_s = ms * 1e-3 / args.steps
    print(f"[bench] {args.steps} steps in {ms:.3f} ms ({avg_launch_s*1e6:.2f} us/step)",
          file=sys.stderr, flush=True)

    last = args.steps - 1
    got = index.cpu().numpy()

    # acceptance of uniform AR on this workload (trials of 32 steps)
    trials = torch.empty(R, dtype=torch.int32, device=dev)
    tsum = nfb = nsel = 0
    for s in range(32):
        arsel.select(bufs[s], M, R, R, arsel.SOA, seed=SEED, step=s, index=index, trials=trials)
        t = trials.cpu().numpy().view(np.uint32).astype(np.int64)
        ok = t <= 4096
        tsum += int(t[ok].sum()) + 4096 * int((~ok).sum())
        nfb += int((~ok).sum())
        nsel += int((t > 0).sum())
    acceptance = {"uniform_per_trial": nsel / tsum if tsum else None,
                  "uniform_mean_trials": tsum / max(nsel, 1),
                  "fallback_fraction": nfb / max(nsel, 1),
                  "learned_per_trial": None}

    bytes_per_launch = R * BYTES_PER_SELECTION
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = load_traffic("select_tile")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}

    print("[bench] read-bandwidth ceiling", file=sys.stderr, flush=True)
    ceiling = bench_ceiling(torch, arsel, bufs)
    best = max(ceiling["contiguous"]["GBs"], ceiling["soa_tile16"]["GBs"])
    roofline["probe_GBs"] = best
    roofline["frac_of_probe"] = round(achieved / best, 4)

    cpu = None
    parity = "not checked (--no-cpu)"
    if not args.no_cpu:
        # all the cores this process may use, at most the box's share of 16
        cores = min(16, host_identity()["usable_cores"] or 1)
        cpu, parity = cpu_baseline(host, threads=cores, last_step=last, gpu_index=got)

    ragged = learned_res = ssa_res = paper_res = scale_res = sens_res = ksweep_res = None
    if not args.no_extras:
        print("[bench] uneven batch", file=sys.stderr, flush=True)
        ragged = bench_ragged(torch, arsel, workloads)
        print("[bench] learned proposal", file=sys.stderr, flush=True)
        learned_res, lp = bench_learned(torch, np, arsel, workloads)
        print("[bench] full SSA run", file=sys.stderr, flush=True)
        ssa_res = bench_ssa(torch, np, arsel, workloads, lp=lp)
        del lp
        print("[bench] paper scheme vs exact AR (Table 1 grid)", file=sys.stderr, flush=True)
        paper_res = bench_paper_table1(torch, np, arsel, workloads)
        print("[bench] selections/s against K for M = 64, 256, 1024", file=sys.stderr, flush=True)
        ksweep_res = bench_k_sweep(torch, np, arsel, workloads)
        print("[bench] 10^6 realizations in one launch", file=sys.stderr, flush=True)
        scale_res = bench_scale(torch)
        print("[bench] sensitivity-analysis shape: 9,261,000 realizations", file=sys.stderr,
              flush=True)
        sens_res = bench_scale(torch, K=9 * 1029 * 1000, reps=3)
        acceptance["learned_per_trial"] = learned_res["per_state"]["acceptance_per_trial"]["learned"]
        acceptance["uniform_per_trial_same_states"] = (
            learned_res["per_state"]["acceptance_per_trial"]["uniform"])

    out = {
        "metric": "next-reaction selections/sec at M=1029 (batched) + AR acceptance rate vs learned q",
        "value": round(sel_per_s, 1), "unit": "selections/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms / args.steps, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched uniform AR: R=4096 realizations x M=1029 reactions, SoA, "
                               "lognormal(0,2) with 30% zeros, 32 rotating batches, one "
                               "selection per realization per step, HIP graph of all steps",
                   "R": R, "M": M, "layout": "SoA", "buffers": NBUF, "seed": SEED},
        "roofline": roofline,
        "read_ceiling": ceiling,
        "cpu_baseline": cpu,
        "acceptance": acceptance,
        "parity_last_step": parity,
        "ragged": ragged,
        "learned": learned_res,
        "ssa_run": ssa_res,
        "paper_table1": paper_res,
        "k_sweep": ksweep_res,
        "scale_1e6": scale_res,
        "sensitivity_9x1029x1000": sens_res,
    }
    print(json.dumps(out), flush=True)
    return 1 if parity.startswith("MISMATCH") else 0


if __name__ == "__main__":
    sys.exit(main())
