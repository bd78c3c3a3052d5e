"""Disorder-chunked runs for batches whose caches do not fit in HBM at once.

Orchestration only: every step of the method runs in the library's kernels
through the C ABI (tnmc_build_env, tnmc_sample, tnmc_energy, tnmc_accept);
this module slices a batch of instances into chunks whose workspace fits a
memory budget, runs the whole path chunk by chunk on one stream, and keeps
each instance's Markov chain and a few running sums.  Every instance's
couplings stay resident in device memory for the whole run (they are small:
8 MB per 1024 x 1024 lattice); the caches of one chunk are built, sampled
and dropped before the next chunk's are built.
"""
from __future__ import annotations

import time

import numpy as np

from . import (CHAIN_BYTES, COUPLING_GENERAL, Problem, chain_state, tnmc_accept, tnmc_build_env,
               tnmc_energy, tnmc_env_check, tnmc_env_stats, tnmc_sample, tnmc_workspace_size)


def plan_chunks(L: int, chi: int, precision: int, n_samples: int, n_inst: int, budget_bytes: float,
                max_chunk: int = 256, flags: int = 0):
    """Largest chunk (at most max_chunk instances) whose workspace and sample
    outputs fit the budget; returns the list of (first, count)."""
    from . import tnmc_workspace_bytes
    per = None
    for k in (1, 2):
        p = Problem(None, None, [L] * k, chi, 1.0, flags=flags)
        b = tnmc_workspace_bytes(p, precision, n_samples)
        if b == 0:
            raise ValueError("bad chunk problem")
        per = b if per is None else b - per
    out_bytes = n_samples * (L * ((L + 63) // 64) * 8 + 8 * 3 + 1)
    size = int(max(1, min(max_chunk, budget_bytes // (per + out_bytes))))
    return [(i, min(size, n_inst - i)) for i in range(0, n_inst, size)]


def run(J_h, J_v, L: int, chi: int, beta: float, precision: int, n_samples: int, seed: int,
        budget_bytes: float = 200e9, coupling_kind: int = COUPLING_GENERAL, max_chunk: int = 256, log=None,
        flags: int = 0):
    """J_h (B, L, L-1), J_v (B, L-1, L): device float32 tensors of every
    instance.  Runs build + n_samples draws + energies + Metropolis chain for
    every instance, chunk by chunk.  Returns a dict with per-instance
    accepted / trial counts, mean energy of the chain states, ln Z, the
    chunk plan and GPU time per phase (hipEvents on the current stream).
    flags are the problem flags (e.g. ALTERNATE_SWEEPS) of every chunk."""
    import torch
    B = J_h.shape[0]
    chunks = plan_chunks(L, chi, precision, n_samples, B, budget_bytes, max_chunk, flags)
    stream = torch.cuda.current_stream()
    n_acc = np.zeros(B, np.int64)
    n_tr = np.zeros(B, np.int64)
    e_mean = np.zeros(B)
    logz = np.zeros(B)
    phase = np.zeros(4)
    t0 = time.perf_counter()
    for (i0, nb) in chunks:
        jh = J_h[i0:i0 + nb]
        jv = J_v[i0:i0 + nb]
        p = Problem(jh, jv, [L] * nb, chi, beta, coupling_kind=coupling_kind, flags=flags)
        ws = torch.empty(tnmc_workspace_size(p, precision, n_samples), dtype=torch.uint8, device="cuda")
        spins = torch.empty(n_samples * p.spin_words_per_sample(), dtype=torch.int64, device="cuda")
        logq = torch.empty((nb, n_samples), dtype=torch.float64, device="cuda")
        E = torch.empty((nb, n_samples), dtype=torch.float64, device="cuda")
        acc = torch.empty((nb, n_samples), dtype=torch.uint8, device="cuda")
        st = torch.empty((nb, n_samples), dtype=torch.int64, device="cuda")
        chain = torch.zeros(nb * CHAIN_BYTES, dtype=torch.uint8, device="cuda")
        bt = torch.full((nb,), float(beta), dtype=torch.float64, device="cuda")
        lz = torch.empty(nb, dtype=torch.float64, device="cuda")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        env = tnmc_build_env(p, precision, ws, lz)
        ev[1].record(stream)
        tnmc_sample(env, n_samples, seed, spins, logq)
        ev[2].record(stream)
        tnmc_energy(p, n_samples, spins, E)
        ev[3].record(stream)
        # the instance index in the accept counter is the chunk-local one;
        # the seed is offset by the chunk's first instance so that chains of
        # different chunks draw from different Philox streams
        tnmc_accept(logq, E, bt, chain, seed + i0, 0, acc, st)
        ev[4].record(stream)
        torch.cuda.synchronize()
        tnmc_env_check(env)
        phase += [ev[k].elapsed_time(ev[k + 1]) * 1e-3 for k in range(4)]
        ch = chain_state(chain.cpu().numpy())
        n_acc[i0:i0 + nb] = [c["n_acc"] for c in ch]
        n_tr[i0:i0 + nb] = [c["n_trials"] for c in ch]
        # mean energy of the chain's states (the Metropolis estimator)
        Eh, sh = E.cpu().numpy(), st.cpu().numpy()
        e_mean[i0:i0 + nb] = np.take_along_axis(Eh, sh, axis=1).mean(axis=1)
        logz[i0:i0 + nb] = lz.cpu().numpy()
        if log:
            log(f"  chunk {i0}..{i0 + nb - 1}: build {ev[0].elapsed_time(ev[1]) / 1e3:.1f} s, sample "
                f"{ev[1].elapsed_time(ev[2]) / 1e3:.1f} s, acceptance {n_acc[i0:i0 + nb].sum() / max(1, n_tr[i0:i0 + nb].sum()):.4f}")
        del env, ws, spins, logq, E, acc, st
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(n_acc=n_acc, n_trials=n_tr, e_mean=e_mean, logz=logz, chunks=chunks, wall_s=wall,
                build_s=phase[0], sample_s=phase[1], energy_s=phase[2], accept_s=phase[3])
