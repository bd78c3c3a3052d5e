"""Schedule autotuner for uneven batches (tnmc_run).

Candidate schedules are timed on a scaled replica of the batch -- the same
mix of bond dimensions, temperatures and coupling families on lattices of
side L / scale -- and the best one for the requested objective is returned.
The candidates:

* one fused launch, longest instance first (shortest whole batch on a full
  machine);
* one fused launch, shortest first (small instances finish early);
* one fused launch per chi bucket (16, 32, 64), each on its own stream:
  smaller buckets need less shared memory per workgroup, so several of
  their workgroups can share a compute unit beside the long builds.

Orchestration only: every measured step runs in the library's kernels; the
per-instance completion times come from the device clock the kernels record
(tnmc_env_stats, 100 MHz ticks).
"""
from __future__ import annotations

import numpy as np

TICKS_PER_S = 1.0e8

CANDIDATES = (
    ("one launch, longest first", "one", 0),
    ("one launch, shortest first", "one", 1),
    ("one launch per chi bucket on its own stream, longest first", "split", 0),
)


def bucket(chi: int) -> int:
    return 16 if chi <= 16 else (32 if chi <= 32 else 64)


def run_schedule(Js, chis, betas, precision: int, n_samples: int, mode: str, order: int,
                 seed: int = 0x5A5A0004):
    """Runs the batch once under one schedule.  Returns a dict: completion
    seconds per instance (input order), wall seconds, accepted and trial
    counts, and the per-instance acceptance."""
    import torch
    from . import (CHAIN_BYTES, Problem, chain_state, tnmc_env_stats, tnmc_run, tnmc_workspace_size)
    B = len(Js)
    Ls = [int(a.shape[0]) for a, _ in Js]
    if mode == "one":
        groups = [list(range(B))]
    else:
        groups = [g for g in ([i for i in range(B) if bucket(chis[i]) == b] for b in (64, 32, 16)) if g]
    cur = torch.cuda.current_stream()
    streams = [cur] if mode == "one" else [torch.cuda.Stream() for _ in groups]
    runs = []
    for g in groups:
        jh = torch.as_tensor(np.concatenate([np.asarray(Js[i][0], np.float32).ravel() for i in g])).cuda()
        jv = torch.as_tensor(np.concatenate([np.asarray(Js[i][1], np.float32).ravel() for i in g])).cuda()
        p = Problem(jh, jv, [Ls[i] for i in g], [chis[i] for i in g], [float(betas[i]) for i in g])
        nb = len(g)
        t = dict(g=g, jh=jh, jv=jv, p=p,
                 ws=torch.empty(tnmc_workspace_size(p, precision, n_samples), dtype=torch.uint8, device="cuda"),
                 spins=torch.empty(n_samples * p.spin_words_per_sample(), dtype=torch.int64, device="cuda"),
                 logq=torch.empty((nb, n_samples), dtype=torch.float64, device="cuda"),
                 E=torch.empty((nb, n_samples), dtype=torch.float64, device="cuda"),
                 acc=torch.empty((nb, n_samples), dtype=torch.uint8, device="cuda"),
                 chain=torch.zeros(nb * CHAIN_BYTES, dtype=torch.uint8, device="cuda"))
        runs.append(t)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for t, s in zip(runs, streams):
        s.wait_event(e0)
        t["env"] = tnmc_run(t["p"], precision, t["ws"], n_samples, seed, t["chain"], seed + 1, t["spins"],
                            t["logq"], t["E"], t["acc"], schedule=order, stream=s)
    for s in streams:
        cur.wait_stream(s)
    e1.record(cur)
    torch.cuda.synchronize()
    start = min(int(tnmc_env_stats(t["env"])[:, 4].min()) for t in runs)
    done = np.zeros(B)
    acc_rate = np.zeros(B)
    n_acc = n_tr = 0
    for t in runs:
        st = tnmc_env_stats(t["env"])
        ch = chain_state(t["chain"].cpu().numpy())
        for k, i in enumerate(t["g"]):
            done[i] = (st[k, 6] - start) / TICKS_PER_S
            acc_rate[i] = ch[k]["n_acc"] / max(1, ch[k]["n_trials"])
            n_acc += ch[k]["n_acc"]
            n_tr += ch[k]["n_trials"]
    return dict(completion_s=done, wall_s=e0.elapsed_time(e1) / 1e3, accepted=n_acc, trials=n_tr,
                acceptance=acc_rate)


def objective_value(res, objective: str) -> float:
    c = res["completion_s"]
    if objective == "p99":
        return float(np.percentile(c, 99))
    if objective == "p50":
        return float(np.percentile(c, 50))
    if objective == "mean":
        return float(c.mean())
    return float(res["wall_s"])      # "makespan"


def tune(instance_fn, spec, precision: int, n_samples: int, objective: str = "p99", scale: int = 4):
    """spec: list of (L, family, chi, beta) per instance; instance_fn(L,
    family, index) -> (J_h, J_v) draws replica couplings.  Returns (best
    candidate name, mode, order, {name: (objective value, result)})."""
    Js = [instance_fn(max(4, L // scale), fam, i) for i, (L, fam, _, _) in enumerate(spec)]
    chis = [c for _, _, c, _ in spec]
    betas = [b for _, _, _, b in spec]
    table = {}
    for name, mode, order in CANDIDATES:
        res = run_schedule(Js, chis, betas, precision, n_samples, mode, order)
        table[name] = (objective_value(res, objective), res)
    best = min(CANDIDATES, key=lambda c: table[c[0]][0])
    return best[0], best[1], best[2], table
