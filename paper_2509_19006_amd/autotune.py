"""Uneven batches (tnmc_run): schedule choice and execution.

The choice is the library's own autotuner (tnmc_autotune, C): candidate
schedules of the persistent pipeline -- one launch in each instance order,
or one launch per bond class on its own stream -- timed on a sub-lattice
replica of the batch, with the answer kept in a tuning cache file.  This
module marshals a batch into one problem, asks the tuner, and runs the
chosen plan on the full batch.

Orchestration only: every measured step runs in the library's kernels; the
per-instance completion times come from the device clock the kernels record
(tnmc_env_stats, 100 MHz ticks).
"""
from __future__ import annotations

import numpy as np

TICKS_PER_S = 1.0e8


def bucket(chi: int) -> int:
    return 16 if chi <= 16 else (32 if chi <= 32 else 64)


def flat_problem(Js, chis, betas, coupling_kind=0):
    """One problem holding every instance (couplings packed in batch order)."""
    import torch
    from . import Problem
    jh = torch.as_tensor(np.concatenate([np.asarray(a, np.float32).ravel() for a, _ in Js])).cuda()
    jv = torch.as_tensor(np.concatenate([np.asarray(b, np.float32).ravel() for _, b in Js])).cuda()
    Ls = [int(a.shape[0]) for a, _ in Js]
    return Problem(jh, jv, Ls, list(chis), [float(b) for b in betas], coupling_kind=coupling_kind)


def tune(Js, chis, betas, precision: int, n_samples: int, objective: str = "p99", scale: int = 4,
         cache_path=None):
    """The library's choice for this batch: dict with schedule, split,
    objective_s, candidates_s (longest-first, shortest-first, as given,
    split by class) and from_cache."""
    from . import tnmc_autotune
    p = flat_problem(Js, chis, betas)
    return tnmc_autotune(p, precision, n_samples, objective, scale, cache_path)


def run_schedule(Js, chis, betas, precision: int, n_samples: int, split: bool, order: int,
                 seed: int = 0x5A5A0004, decode_steps: int = 0):
    """Runs the batch once under one plan: one tnmc_run in `order`, or (split)
    one tnmc_run per bond class, each on its own stream, longest-first.
    Returns a dict: completion seconds per instance (input order), wall
    seconds, accepted and trial counts, and the per-instance acceptance.

    With decode_steps > 0 the built caches are then reused: that many
    further decode steps per instance (tnmc_sample, tnmc_energy, tnmc_accept
    of n_samples fresh draws, the chains continuing) are captured once into
    a HIP graph and replayed; their accepted / trial counts and wall time
    are returned under "decode"."""
    import torch
    from . import (CHAIN_BYTES, Problem, chain_state, tnmc_env_stats, tnmc_run, tnmc_workspace_size)
    B = len(Js)
    Ls = [int(a.shape[0]) for a, _ in Js]
    if not split:
        groups = [list(range(B))]
    else:
        groups = [g for g in ([i for i in range(B) if bucket(chis[i]) == b] for b in (64, 32, 16)) if g]
    cur = torch.cuda.current_stream()
    streams = [cur] if not split else [torch.cuda.Stream() for _ in groups]
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
                            t["logq"], t["E"], t["acc"], schedule=order if not split else 0, stream=s)
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
    out = dict(completion_s=done, wall_s=e0.elapsed_time(e1) / 1e3, accepted=n_acc, trials=n_tr,
               acceptance=acc_rate)
    if decode_steps > 0:
        out["decode"] = _graph_decode(runs, precision, n_samples, seed, decode_steps)
    return out


def _graph_decode(runs, precision, n_samples, seed, steps):
    """Decode steps on the built caches, captured into one HIP graph."""
    import torch
    from . import chain_state, tnmc_accept, tnmc_energy, tnmc_sample
    for t in runs:
        t["beta_t"] = torch.as_tensor(np.asarray(t["p"].beta, np.float64)).cuda()
        t["n0"] = sum(c["n_acc"] for c in chain_state(t["chain"].cpu().numpy()))
        t["t0"] = sum(c["n_trials"] for c in chain_state(t["chain"].cpu().numpy()))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for k in range(1, steps + 1):
                off = k * n_samples
                for t in runs:
                    tnmc_sample(t["env"], n_samples, seed, t["spins"], t["logq"], sample_offset=off, stream=s)
                    tnmc_energy(t["p"], n_samples, t["spins"], t["E"], stream=s)
                    tnmc_accept(t["logq"], t["E"], t["beta_t"], t["chain"], seed + 1, off, t["acc"], stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    acc = tr = 0
    for t in runs:
        st = chain_state(t["chain"].cpu().numpy())
        acc += sum(c["n_acc"] for c in st) - t["n0"]
        tr += sum(c["n_trials"] for c in st) - t["t0"]
    return dict(steps=steps, accepted=acc, trials=tr, wall_s=e0.elapsed_time(e1) / 1e3)
