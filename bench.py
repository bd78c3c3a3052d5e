#!/usr/bin/env python3
"""Throughput of the batched TNMC hot path on one MI355X.

One step = the whole path over one batch of synthetic disorders: boundary-MPS
cache build (tnmc_build_env), sampling (tnmc_sample), exact energies
(tnmc_energy, float64 and int32) and the Metropolis independence step
(tnmc_accept), all on one stream with the couplings already resident in HBM.
Default workload: 256 x 256 open-boundary +-J Edwards-Anderson lattices,
beta = 1, chi = 32, 256 disorders x 256 samples, run through the plain
float32 path (the headline value) and through the float16-stored-cache form
on the same inputs.  The Markov chains continue across steps; accepted
samples are accepted Metropolis trials.

Prints one JSON line with the headline value, both forms, a roofline entry
for the dominant kernel (the cache build) and one per form for the sampler,
and the CPU oracle run end to end on one instance of the workload in a child
process while the GPU forms run.

Other workloads (--workload): uneven (the 512-instance mix in one persistent
launch), learned (the learned proposal correction), paper (the paper's
1024 x 1024 +-J run at chi = 8, disorder-chunked) and sweep (acceptance
against L, chi and beta).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

METRIC = "accepted samples/s at L=256 chi=32 + acceptance rate, learned/mixed vs plain"
# MI355X published peaks: vector float32 / float64 flop/s, dense bf16/fp16
# MFMA flop/s, HBM bytes/s
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12, "mfma16": 2.5e15, "hbm": 8.0e12}

# HBM bytes per launch at the default workload (256 x 256, chi 32, 256 x 256)
# from two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE), each scaled by
# what the same counter reads for a plain device copy of known size; valid
# only for the kernel source they were measured on (sha256 over the files
# listed), reported as null otherwise.
TRAFFIC_PROFILE = "profiles/k_build_k_sample_mfma_256x256_chi32_hbm_traffic.txt"
TRAFFIC = {
    "k_build": {"sources": ["paper_2509_19006_amd/csrc/build.hip", "paper_2509_19006_amd/csrc/build_device.hpp",
                            "paper_2509_19006_amd/csrc/build_pipe.hpp", "paper_2509_19006_amd/csrc/device.hpp"],
                "sha256": "3ebafc8986e3c2de88c256c5a3addda6e41558d7c82014998a7040040b3cac13",
                "sweeps": "alternating",
                "bytes": {"fp32": 863431011740, "bf16x3": 863431011740,
                          "fp16": 781035878871}},
    "k_sample_mfma": {"sources": ["paper_2509_19006_amd/csrc/sample.hip", "paper_2509_19006_amd/csrc/sample_mfma.hpp",
                                  "paper_2509_19006_amd/csrc/device.hpp"],
                      "sha256": "a278a128d862b30f01e185037317bfba4acf0034e23a2771556e3b82fdb4a25e",
                      "bytes": {"fp32": 1388365171118, "bf16x3": 1388213535742,
                                "fp16": 1250854359868}},
}


def traffic_for(kernel, form, sweeps=None):
    """Counter-measured HBM bytes of one launch of kernel in the given form
    (and, for the build, sweep order), or None when the kernel's source has
    changed since the measurement."""
    import hashlib
    ent = TRAFFIC.get(kernel)
    if ent is None or form not in ent["bytes"]:
        return None
    if "sweeps" in ent and sweeps != ent["sweeps"]:
        return None
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in ent["sources"]:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return ent["bytes"][form] if h.hexdigest() == ent["sha256"] else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_flops_dense(L, chi, B):
    """Flops of one cache build under the dense boundary-MPS cost model: per
    site of every row above the bottom one, 32 chi^2 + (101 + 48 S) chi^3
    with S = 8 Jacobi sweeps (dense MPO apply, 4chi x 2chi QR with explicit
    Q, 2chi x 2chi one-sided Jacobi).  A reference figure only: the kernel
    does not execute this work."""
    per_site = 32 * chi ** 2 + (101 + 48 * 8) * chi ** 3
    return B * (L - 1) * L * per_site


def build_flops_executed(L, chi, B, sweeps_per_site):
    """Flops the spin-flip (Z2) symmetric kernel executes in one cache build:
    per bulk site-row two parity blocks, each a 2chi x chi Householder QR with
    its explicit Q (2 x 10/3 chi^3), the carried-R product of a chi x chi by
    a chi x 2chi block (4 chi^3), the chi x chi centre T = Q X (2 chi^3) and
    the one-sided Jacobi on a chi x chi block at 7 chi^3 per sweep (chi^2/2
    pairs, each one dot product and two column rotations of length chi plus
    the two rotated columns of W); with S the measured sweeps per site this
    is (2 chi^2 +) (25.3 + 14 S) chi^3 per site-row, the O(chi^2) apply
    included."""
    per_site = 2 * chi ** 2 + (2 * (20.0 / 3 + 4 + 2)) * chi ** 3 + 14.0 * sweeps_per_site * chi ** 3
    return B * (L - 1) * L * per_site


def sample_flops(L, chi, B, N):
    """Algorithmic flops of one sampling pass: 8 chi^2 per site-sample (left
    product l A_s for both spins and the right-environment product, 2 chi^2
    multiply-adds each)."""
    return 8 * chi ** 2 * L * L * B * N


def sample_bytes(L, chi, B, N, cache_elem_bytes):
    """Algorithmic HBM bytes of one sampling pass: the cache read once
    (2 chi^2 entries per site) and the packed spins written once."""
    return B * L * L * 2 * chi ** 2 * cache_elem_bytes + B * N * L * ((L + 63) // 64) * 8


def run_form(T, torch, prec, jh, jv, L, chi, beta, B, N, steps, warmup, seed, flags=0):
    problem = T.Problem(jh, jv, [L] * B, chi, beta, coupling_kind=T.COUPLING_PMJ, flags=flags)
    nbytes = T.tnmc_workspace_size(problem, prec, N)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    words = N * problem.spin_words_per_sample()
    spins = torch.empty(words, dtype=torch.int64, device="cuda")
    logq = torch.empty((B, N), dtype=torch.float64, device="cuda")
    E = torch.empty((B, N), dtype=torch.float64, device="cuda")
    E_int = torch.empty((B, N), dtype=torch.int32, device="cuda")
    acc = torch.empty((B, N), dtype=torch.uint8, device="cuda")
    chain = torch.zeros(B * T.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
    beta_t = torch.full((B,), float(beta), dtype=torch.float64, device="cuda")
    logz = torch.empty(B, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    envs = []

    def step(k, marks=None):
        if marks: marks[0].record(stream)
        env = T.tnmc_build_env(problem, prec, ws, logz)
        if marks: marks[1].record(stream)
        T.tnmc_sample(env, N, seed, spins, logq, sample_offset=k * N)
        if marks: marks[2].record(stream)
        T.tnmc_energy(problem, N, spins, E, E_int)
        if marks: marks[3].record(stream)
        T.tnmc_accept(logq, E, beta_t, chain, seed, k * N, acc)
        if marks: marks[4].record(stream)
        envs.append(env)

    for w in range(warmup):
        step(10_000 + w)
        torch.cuda.synchronize()
        log(f"  warmup step {w} done")
    chain.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k, ev[k])
        torch.cuda.synchronize()
        log(f"  step {k}: build {ev[k][0].elapsed_time(ev[k][1]):.0f} ms, "
            f"sample {ev[k][1].elapsed_time(ev[k][2]):.0f} ms")
    wall = time.perf_counter() - t0
    st = T.chain_state(chain.cpu().numpy())
    n_acc = sum(s["n_acc"] for s in st)
    n_tr = sum(s["n_trials"] for s in st)
    phase = [sum(ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(steps)) / steps for i in range(4)]
    stats = T.tnmc_env_stats(envs[-1])
    T.tnmc_env_check(envs[-1])           # raises on a non-finite log-scale / unconverged Jacobi
    assert torch.equal(E_int.double(), E), "int32 and float64 energies differ"
    out = dict(value=n_acc / wall, acceptance=n_acc / max(1, n_tr), accepted=n_acc, trials=n_tr,
               wall_s=wall, ms_per_step=1e3 * wall / steps,
               build_ms=phase[0], sample_ms=phase[1], energy_ms=phase[2], accept_ms=phase[3],
               # the rate once a built cache is reused for further batches of
               # proposals (no rebuild): sampling, energies and accept only
               accepted_per_s_cache_reused=n_acc / (steps * 1e-3 * (phase[1] + phase[2] + phase[3])),
               jacobi_sweeps_per_site=float(stats[:, 0].mean()) / ((L - 1) * L),
               build_phase_share=build_phase_share(stats),
               mean_energy_per_spin=float(E.mean().item()) / (L * L),
               logz_mean=float(logz.mean().item()))
    del envs, ws
    torch.cuda.empty_cache()
    return out


def build_phase_share(stats):
    """Shares of an instance's build time (device wall clock, averaged over
    instances) spent in the QR sweep (of it, the Householder
    factorisations) and in the SVD sweep (of it, the Jacobi)."""
    import numpy as np
    st = np.asarray(stats, dtype=np.float64)
    tot = np.maximum(st[:, 5] - st[:, 4], 1.0)
    share = lambda i: round(float((st[:, i] / tot).mean()), 4)
    return {"qr_sweep": share(1), "householder": share(7), "svd_sweep": share(2), "jacobi": share(3)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# the oracle leg runs on a smaller lattice of the same family (same chi,
# beta and coupling distribution) so that it stays at a few tens of seconds
# of host work; its rate is scaled to the workload's side by the number of
# site-rows, which sets the cost of both the cache build and a draw
CPU_SAMPLE_L = 96


def cpu_baseline_child(L, chi, beta, n_sample, L_full, alternate=False):
    """The oracle end to end on one instance (the first disorder of a batch
    of side L): the float64 cache build of all L - 1 rows, n_sample draws,
    their energies and the Metropolis chain over them.  Prints progress to
    stderr and one JSON line to stdout; runs in a child process beside the
    GPU forms."""
    import numpy as np
    import workloads
    from oracle import bmps, ising, mis, sampler
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = len(os.sched_getaffinity(0))
    jh, jv = workloads.batch(L, 1, "pmj", 3)
    jh, jv = jh[0].astype(np.float64), jv[0].astype(np.float64)
    t0 = time.perf_counter()
    cache, _, _ = bmps.build_cache(beta, jh, jv, chi, alternate=alternate)
    t_build = time.perf_counter() - t0
    log(f"  oracle leg: cache build of {L - 1} rows done ({t_build:.1f} s)")
    bits, logq, _ = sampler.sample(cache, beta, jv, n_sample, seed=0x5A5A0003)
    E = ising.energy(2 * bits - 1, jh, jv)
    chain = mis.Chain()
    mis.accept(logq, E, beta, chain, 0x5A5A0003, 0, 0)
    wall = time.perf_counter() - t0
    log(f"  oracle leg: {n_sample} draws and the chain done ({wall:.1f} s)")
    rate = chain.n_acc / wall
    scale = (L * (L - 1)) / (L_full * (L_full - 1))
    print(json.dumps({"value": rate * scale, "unit": "accepted samples/s", "cores": int(cores),
                      "kind": "oracle", "cpu": cpu_model(),
                      "value_at_sample_size": rate, "scale_to_workload": scale,
                      "acceptance": chain.n_acc / max(1, chain.n_trials), "trials": chain.n_trials,
                      "wall_s": wall, "build_s": t_build,
                      "sample": (f"one {L}x{L} +-J instance of the workload's family (chi={chi}, beta={beta}): "
                                 f"the float64 cache build of all {L - 1} rows ({'alternating' if alternate else 'plain'} "
                                 f"sweep order) ({t_build:.1f} s), {n_sample} "
                                 f"draws, their energies and the oracle's own Metropolis chain "
                                 f"({chain.n_acc} of {chain.n_trials} trials accepted), timed end to end; "
                                 f"the rate scaled to {L_full}x{L_full} by the site-row ratio "
                                 f"{L}*{L - 1}/({L_full}*{L_full - 1})")}),
          flush=True)


def start_cpu_baseline(L, chi, beta, n_sample=8, alternate=False):
    """Starts the oracle leg as a child process before this process touches
    the GPU; collect it with finish_cpu_baseline."""
    import subprocess
    Ls = min(L, CPU_SAMPLE_L)
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--L", str(Ls), "--chi", str(chi),
           "--beta", str(beta), "--samples", str(n_sample), "--full-L", str(L),
           "--sweeps", "alternating" if alternate else "plain"]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True)


def finish_cpu_baseline(proc, timeout_s=240):
    import subprocess
    log("waiting for the oracle leg")
    try:
        out, _ = proc.communicate(timeout=timeout_s)
    except subprocess.TimeoutExpired:
        proc.kill()
        proc.communicate()
        log(f"oracle leg still running after {timeout_s} s more: stopped, no cpu baseline")
        return None
    if proc.returncode != 0:
        log(f"cpu baseline failed with status {proc.returncode}")
        return None
    return json.loads(out.strip().splitlines()[-1])


def c4_spec():
    """The uneven batch: 512 instances, L in {32, 64, 128, 256} (equal
    counts), +-J when floor(i/4) is even else Gaussian, chi in {16, 32, 64}
    by floor(i/8) mod 3, beta uniform in [0.5, 2.0]."""
    import workloads
    betas = workloads.betas_uniform(512, 0.5, 2.0, 4)
    return [((32, 64, 128, 256)[i % 4], "pmj" if (i // 4) % 2 == 0 else "gauss",
             (16, 32, 64)[(i // 8) % 3], float(betas[i])) for i in range(512)]


def run_uneven(args):
    """Uneven batch in one persistent launch per schedule; the schedule comes
    from the autotuner (candidates timed on a 1/4-scale replica)."""
    import numpy as np
    import paper_2509_19006_amd as T
    from paper_2509_19006_amd import autotune
    import workloads
    T.load()
    spec = c4_spec()
    N = 32
    Js = [workloads.instance(L, fam, 4, i) for i, (L, fam, _, _) in enumerate(spec)]
    chis = [c for _, _, c, _ in spec]
    betas = [b for _, _, _, b in spec]
    log(f"uneven batch: {len(spec)} instances, {N} samples each; the library's tuner times the candidate "
        f"schedules on a 1/4-scale sub-lattice replica (objective {args.objective})")
    import tempfile
    cache = os.path.join(tempfile.gettempdir(), "tnmc_tuning.txt")
    tune = autotune.tune(Js, chis, betas, T.FP32, N, objective=args.objective, scale=4, cache_path=cache)
    cands = ["longest-first", "shortest-first", "as given", "split by bond class"]
    for k, v in zip(cands, tune["candidates_s"]):
        log(f"  {k}: {args.objective} {v:.3f} s (replica)")
    name = cands[3] if tune["split"] else cands[tune["schedule"]]
    log(f"chosen: {name}{' (from the tuning cache)' if tune['from_cache'] else ''}; full batch ...")
    res = autotune.run_schedule(Js, chis, betas, T.FP32, N, tune["split"], tune["schedule"], decode_steps=4)
    dec = res["decode"]
    log(f"  then 4 decode steps per instance from one captured graph: {dec['wall_s']:.2f} s, acceptance "
        f"{dec['accepted'] / max(1, dec['trials']):.4f}")
    c = res["completion_s"]
    by_class = {}
    for (L, _, chi, _), t in zip(spec, c):
        by_class.setdefault(f"L{L}_chi{chi}", []).append(t)
    line = {
        "metric": "accepted samples/s, uneven batch in one persistent launch, + p50/p99 per-instance completion",
        "value": res["accepted"] / res["wall_s"], "unit": "accepted samples/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": res["wall_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uneven batch: 512 instances, L in {32,64,128,256}, half +-J half Gaussian, "
                               "beta in [0.5, 2], chi in {16,32,64}, 32 samples each, float32",
                   "schedule": name, "objective": args.objective},
        "proposals_per_s": len(spec) * N / res["wall_s"],
        "acceptance": res["accepted"] / max(1, res["trials"]),
        "completion_p50_s": float(np.percentile(c, 50)), "completion_p99_s": float(np.percentile(c, 99)),
        "completion_max_s": float(c.max()),
        "completion_median_by_class_s": {k: float(np.median(v)) for k, v in sorted(by_class.items())},
        "tuner_replica_objective_s": dict(zip(cands, tune["candidates_s"])),
        "graph_decode": {"steps_per_instance": dec["steps"], "samples_per_step": N, "wall_s": dec["wall_s"],
                         "accepted": dec["accepted"], "trials": dec["trials"],
                         "accepted_per_s_cache_reused": dec["accepted"] / dec["wall_s"]},
    }
    print(json.dumps(line), flush=True)


def run_learned(args):
    """Learned-correction form: a chi = 16 proposal whose per-site logits are
    corrected by the MLP, trained on the GPU on chi = 64 conditionals of 16
    separately seeded 256 x 256 Gaussian disorders (one trajectory each,
    about 10^6 sites, spin-flip augmented), against the plain chi = 16 and
    chi = 32 proposals on 1024 x 1024 Gaussian disorders at beta = 1."""
    import numpy as np
    import torch
    import paper_2509_19006_amd as T
    from paper_2509_19006_amd import learned
    import workloads
    T.load()
    beta, Lt, L, B, N, B32 = 1.0, args.train_L, args.L, args.disorders, args.samples, args.disorders_chi32
    t0 = time.time()
    train_J = [workloads.instance(Lt, "gauss", 50, i) for i in range(16)]
    log(f"training data: 16 disorders of {Lt}x{Lt}, chi 16 scored on chi 64 draws ...")
    feat, lo, tgt = learned.make_training_data(train_J, 16, 64, beta, 1, seed=5)
    torch.cuda.synchronize()
    t_data = time.time() - t0
    log(f"  {lo.numel()} rows in {t_data:.1f} s; training {args.train_steps} Adam steps ...")
    t1 = time.time()
    P, losses = learned.train(feat, lo, tgt, steps=args.train_steps, batch=8192, lr=1e-3, seed=1, log=log)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    del feat, lo, tgt
    torch.cuda.empty_cache()

    def form(chi, nb, mlps):
        Js = [workloads.instance(L, "gauss", 5, i) for i in range(nb)]
        jh = torch.as_tensor(np.concatenate([a.ravel() for a, _ in Js])).cuda()
        jv = torch.as_tensor(np.concatenate([b.ravel() for _, b in Js])).cuda()
        p = T.Problem(jh, jv, [L] * nb, chi, beta)
        ws = torch.empty(T.tnmc_workspace_size(p, T.FP32, N), dtype=torch.uint8, device="cuda")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        env = T.tnmc_build_env(p, T.FP32, ws)
        ev[1].record()
        torch.cuda.synchronize()
        build_s = ev[0].elapsed_time(ev[1]) / 1e3
        out = {}
        for name, m in mlps:
            spins = torch.empty(N * p.spin_words_per_sample(), dtype=torch.int64, device="cuda")
            logq = torch.empty((nb, N), dtype=torch.float64, device="cuda")
            E = torch.empty((nb, N), dtype=torch.float64, device="cuda")
            acc = torch.empty((nb, N), dtype=torch.uint8, device="cuda")
            chain = torch.zeros(nb * T.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
            bt = torch.full((nb,), beta, dtype=torch.float64, device="cuda")
            e2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e2[0].record()
            T.tnmc_sample(env, N, 0x5A5A0005, spins, logq, mlp=m)
            T.tnmc_energy(env, N, spins, E)
            T.tnmc_accept(logq, E, bt, chain, 0x5A5A0005, 0, acc)
            e2[1].record()
            torch.cuda.synchronize()
            st = T.chain_state(chain.cpu().numpy())
            na = sum(c["n_acc"] for c in st)
            nt = sum(c["n_trials"] for c in st)
            samp_s = e2[0].elapsed_time(e2[1]) / 1e3
            out[name] = {"chi": chi, "disorders": nb, "acceptance": na / max(1, nt), "accepted": na, "trials": nt,
                         "build_s": build_s, "sample_energy_accept_s": samp_s,
                         "accepted_per_s": na / (build_s + samp_s)}
            log(f"  {name}: acceptance {na / max(1, nt):.4f}, build {build_s:.1f} s, sampling {samp_s:.2f} s")
        del ws, env
        torch.cuda.empty_cache()
        return out

    log(f"evaluation: {B} Gaussian disorders of {L}x{L}, {N} samples, beta {beta}")
    res = form(16, B, [("plain chi16", None), ("learned chi16+mlp", P)])
    log(f"plain chi 32 on {B32} of the disorders ...")
    res.update(form(32, B32, [("plain chi32", None)]))
    lr = res["learned chi16+mlp"]
    line = {
        "metric": "accepted samples/s + acceptance rate, learned correction vs plain",
        "value": lr["accepted_per_s"], "unit": "accepted samples/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": (lr["build_s"] + lr["sample_energy_accept_s"]) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"learned-correction TNMC: {L}x{L} Gaussian lattices, beta 1, {B} disorders x {N} "
                               f"samples; chi 16 + 3-layer MLP (width 64, bf16 weights) trained on chi 64 "
                               f"conditionals of 16 separately seeded {Lt}x{Lt} disorders"},
        "forms": res,
        "training": {"rows": int(2 * 16 * Lt * Lt), "data_s": t_data, "train_s": t_train,
                     "steps": args.train_steps, "loss_first_last": [losses[0][1], losses[-1][1]]},
    }
    print(json.dumps(line), flush=True)


# The paper's single-GPU run (+-J EA, 1024 x 1024, beta 1, chi 8, 10^3
# disorders x 10^3 samples): 3.3 h at acceptance ~0.37, i.e. 10^6 proposals in
# 11 880 s, 0.37 * 10^6 / 11 880 = 31.1 accepted samples/s, on a GPU whose
# model the paper does not state.
PAPER_SECONDS = 3.3 * 3600
PAPER_ACCEPTED_PER_S = 0.37 * 1e6 / PAPER_SECONDS


def run_paper(args):
    """The paper's run: +-J EA lattices of 1024 x 1024 at beta 1, chi 8,
    every disorder's couplings resident in HBM, the disorders processed in
    chunks whose caches fit the memory budget (float32 path)."""
    import numpy as np
    import torch
    import paper_2509_19006_amd as T
    from paper_2509_19006_amd import chunked
    import workloads
    T.load()
    L, chi, B, N, beta = args.L, args.chi, args.disorders, args.samples, args.beta
    log(f"paper workload: {B} +-J disorders of {L}x{L}, beta {beta}, chi {chi}, {N} samples each")
    t0 = time.time()
    jh = torch.empty((B, L, L - 1), dtype=torch.float32, device="cuda")
    jv = torch.empty((B, L - 1, L), dtype=torch.float32, device="cuda")
    for i in range(B):
        a, b = workloads.instance(L, "pmj", 8, i)
        jh[i].copy_(torch.from_numpy(a))
        jv[i].copy_(torch.from_numpy(b))
    torch.cuda.synchronize()
    log(f"  couplings generated and uploaded in {time.time() - t0:.0f} s (not timed)")
    res = chunked.run(jh, jv, L, chi, beta, T.FP32, N, 0x5A5A0008, budget_bytes=args.budget_gb * 1e9,
                      coupling_kind=T.COUPLING_PMJ, log=log,
                      flags=T.ALTERNATE_SWEEPS if args.sweeps == "alternating" else 0)
    acc, tr = int(res["n_acc"].sum()), int(res["n_trials"].sum())
    per_inst = res["n_acc"] / np.maximum(1, res["n_trials"])
    value = acc / res["wall_s"]
    line = {
        "metric": "accepted samples/s + acceptance rate, the paper's 1024x1024 +-J run",
        "value": value, "unit": "accepted samples/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": res["wall_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": value / PAPER_ACCEPTED_PER_S, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"paper run: {B} +-J EA disorders of {L}x{L}, beta {beta}, chi {chi}, {N} samples "
                               f"each, float32, {args.sweeps} sweep order, disorders in chunks of "
                               f"{res['chunks'][0][1]}"},
        "acceptance": acc / max(1, tr),
        "acceptance_per_disorder_mean_sd": [float(per_inst.mean()), float(per_inst.std(ddof=1)) if B > 1 else 0.0],
        "wall_s": res["wall_s"], "build_s": res["build_s"], "sample_s": res["sample_s"],
        "energy_s": res["energy_s"], "accept_s": res["accept_s"],
        "energy_per_spin_chain_mean": float(res["e_mean"].mean() / (L * L)),
        "proposals_per_s": B * N / res["wall_s"],
        "paper": {"seconds": PAPER_SECONDS, "acceptance": 0.37, "accepted_per_s": PAPER_ACCEPTED_PER_S,
                  "hardware": "one GPU, model not stated", "speedup_wall": PAPER_SECONDS * (B * N / 1e6) / res["wall_s"]},
    }
    print(json.dumps(line), flush=True)


def run_sweep(args):
    """Acceptance against L, chi and beta on +-J EA lattices (the paper's
    acceptance figure): per L, every (chi, beta, disorder) combination as one
    uneven batch in one persistent launch (tnmc_run, float32), 16 disorders
    x 64 samples each."""
    import numpy as np
    import torch
    import paper_2509_19006_amd as T
    import workloads
    T.load()
    Ls = [8, 16, 32, 64, 128, 256, 512, 1024]
    chis = [2, 4, 8, 16, 32]
    betas = [0.66, 1.0, 1.5]
    D, N = 16, 64
    table = []
    t0 = time.time()
    for L in Ls:
        combos = [(chi, beta) for chi in chis for beta in betas if not (L >= 1024 and chi > 16)]
        inst = [(chi, beta, d) for chi, beta in combos for d in range(D)]
        Js = [workloads.instance(L, "pmj", 9, d) for d in range(D)]
        jh = torch.as_tensor(np.concatenate([Js[d][0].ravel() for _, _, d in inst])).cuda()
        jv = torch.as_tensor(np.concatenate([Js[d][1].ravel() for _, _, d in inst])).cuda()
        p = T.Problem(jh, jv, [L] * len(inst), [c for c, _, _ in inst], [b for _, b, _ in inst],
                      coupling_kind=T.COUPLING_PMJ)
        B = len(inst)
        ws = torch.empty(T.tnmc_workspace_size(p, T.FP32, N), dtype=torch.uint8, device="cuda")
        spins = torch.empty(N * p.spin_words_per_sample(), dtype=torch.int64, device="cuda")
        lq = torch.empty((B, N), dtype=torch.float64, device="cuda")
        E = torch.empty((B, N), dtype=torch.float64, device="cuda")
        acc = torch.empty((B, N), dtype=torch.uint8, device="cuda")
        chain = torch.zeros(B * T.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
        t1 = time.time()
        env = T.tnmc_run(p, T.FP32, ws, N, 0x5A5A0009, chain, 0x5A5A000A, spins, lq, E, acc)
        torch.cuda.synchronize()
        T.tnmc_env_check(env)
        wall = time.time() - t1
        undefined_logz = int(T.tnmc_env_stats(env)[:, T.STAT_LOGZ_UNDEFINED].sum())
        st = T.chain_state(chain.cpu().numpy())
        a = np.array([c["n_acc"] / max(1, c["n_trials"]) for c in st])
        for k, (chi, beta) in enumerate(combos):
            ak = a[k * D:(k + 1) * D]
            table.append({"L": L, "chi": chi, "beta": beta, "acceptance": float(ak.mean()),
                          "sd_over_disorders": float(ak.std(ddof=1)), "wall_s_launch": wall})
        if undefined_logz:
            log(f"  L {L}: {undefined_logz} instance(s) with an undefined ln Z estimate (truncated total <= 0)")
        log(f"  L {L:5d}: {B} instances in one launch, {wall:.1f} s; acceptance by (chi, beta): " +
            ", ".join(f"{chi}/{beta}: {a[k * D:(k + 1) * D].mean():.3f}" for k, (chi, beta) in enumerate(combos)))
        del env, ws, spins, lq, E, acc, chain, jh, jv
        torch.cuda.empty_cache()
    line = {"metric": "acceptance rate against L, chi and beta (+-J EA, 16 disorders x 64 samples)",
            "value": None, "unit": "acceptance", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": (time.time() - t0) * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "acceptance sweep: L in 8..1024, chi in 2..32 (to 16 at 1024), "
                                   "beta in {0.66, 1, 1.5}, one uneven launch per L"},
            "table": table}
    print(json.dumps(line), flush=True)


def run_rbim(args):
    """Random-bond Ising model along the Nishimori line: for each
    antiferromagnetic fraction p, beta_N = ln((1-p)/p)/2, 64 disorders of
    32 x 32 at chi 16 (float32), two independent chains of 256 proposals per
    disorder.  Reports the disorder-averaged energy per bond of the chain
    states against the exact -tanh(beta_N), the replica-overlap moments
    [<q^2>], [<q^4>] and the Binder ratio, and the acceptance."""
    import numpy as np
    import torch
    import paper_2509_19006_amd as T
    import workloads
    T.load()
    L, chi, D, N = 32, 16, 64, 256
    rows = []
    t0 = time.time()
    for pr in (0.05, 0.1, 0.15, 0.2, 0.25):
        beta = 0.5 * math.log((1 - pr) / pr)
        Js = [workloads.instance(L, "pmj", 12, d, p=pr) for d in range(D)]
        jh = torch.as_tensor(np.stack([a for a, _ in Js])).cuda()
        jv = torch.as_tensor(np.stack([b for _, b in Js])).cuda()
        prob = T.Problem(jh, jv, [L] * D, chi, beta, coupling_kind=T.COUPLING_PMJ)
        ws = torch.empty(T.tnmc_workspace_size(prob, T.FP32, N), dtype=torch.uint8, device="cuda")
        env = T.tnmc_build_env(prob, T.FP32, ws)
        bt = torch.full((D,), beta, dtype=torch.float64, device="cuda")
        sp, st, en, na, ntr = [], [], [], 0, 0
        for chain_seed in (0x5A5A0012, 0x5A5A0013):
            spins = torch.empty(N * prob.spin_words_per_sample(), dtype=torch.int64, device="cuda")
            lq = torch.empty((D, N), dtype=torch.float64, device="cuda")
            E = torch.empty((D, N), dtype=torch.float64, device="cuda")
            acc = torch.empty((D, N), dtype=torch.uint8, device="cuda")
            state = torch.empty((D, N), dtype=torch.int64, device="cuda")
            chain = torch.zeros(D * T.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
            T.tnmc_sample(env, N, chain_seed, spins, lq)
            T.tnmc_energy(prob, N, spins, E)
            T.tnmc_accept(lq, E, bt, chain, chain_seed, 0, acc, state)
            sp.append(spins)
            st.append(state)
            en.append(torch.gather(E, 1, state))
            c = T.chain_state(chain.cpu().numpy())
            na += sum(x["n_acc"] for x in c)
            ntr += sum(x["n_trials"] for x in c)
        q = torch.empty((D, N), dtype=torch.float64, device="cuda")
        T.tnmc_overlap(prob, N, sp[0], st[0], sp[1], st[1], q)
        torch.cuda.synchronize()
        T.tnmc_env_check(env)
        nb = 2 * L * (L - 1)
        e = torch.cat(en, 1).mean(1).cpu().numpy() / nb            # per disorder, per bond
        qh = q.cpu().numpy()
        q2 = (qh ** 2).mean(1)
        q4 = (qh ** 4).mean(1)
        rows.append({"p": pr, "beta_N": beta, "energy_per_bond": float(e.mean()),
                     "energy_per_bond_err": float(e.std(ddof=1) / math.sqrt(D)),
                     "exact_energy_per_bond": -math.tanh(beta),
                     "q2": float(q2.mean()), "q4": float(q4.mean()),
                     "binder": float(0.5 * (3.0 - q4.mean() / q2.mean() ** 2)),
                     "acceptance": na / max(1, ntr)})
        log(f"  p {pr:.2f} (beta_N {beta:.3f}): energy/bond {e.mean():.5f} +- {e.std(ddof=1) / math.sqrt(D):.5f} "
            f"(exact {-math.tanh(beta):.5f}), [<q^2>] {q2.mean():.4f}, Binder {rows[-1]['binder']:.3f}, "
            f"acceptance {rows[-1]['acceptance']:.4f}")
        del env, ws
    line = {"metric": "Nishimori-line RBIM observables (energy per bond vs exact, replica overlap)",
            "value": None, "unit": "energy per bond", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": (time.time() - t0) * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"RBIM on the Nishimori line, {D} disorders of {L}x{L}, chi {chi}, "
                                   f"two chains x {N} proposals"},
            "table": rows}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=None, help="lattice side (headline 256, paper 1024)")
    ap.add_argument("--chi", type=int, default=None, help="bond dimension (headline 32, paper 8)")
    ap.add_argument("--disorders", type=int, default=None, help="disorders (headline 256, paper 1000)")
    ap.add_argument("--samples", type=int, default=None, help="samples per disorder (headline 256, paper 1000)")
    ap.add_argument("--beta", type=float, default=1.0)
    ap.add_argument("--budget-gb", type=float, default=200.0,
                    help="paper / sweep: device memory for one chunk of disorders")
    ap.add_argument("--forms", default="fp32,bf16x3,fp16",
                    help="precision forms of the headline workload, comma separated (the first is fp32): "
                         "fp32, bf16x3, fp16, bf16")
    ap.add_argument("--sweeps", choices=["alternating", "plain"], default="alternating",
                    help="compression sweep order of the cache build: alternating (every second row "
                         "mirrored; float builds with chi <= 32 then pipeline their rows) or plain")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--full-L", type=int, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["headline", "uneven", "learned", "paper", "sweep", "rbim"],
                    default="headline",
                    help="headline: the 256x256 batch (default); uneven: the 512-instance mix in one "
                         "persistent launch with an autotuned schedule; learned: the learned correction "
                         "(use with --L 1024 --disorders 64 --samples 16)")
    ap.add_argument("--train-L", type=int, default=256, help="learned: side of the training lattices")
    ap.add_argument("--train-steps", type=int, default=1500, help="learned: Adam steps")
    ap.add_argument("--disorders-chi32", type=int, default=16, help="learned: disorders of the chi 32 comparison")
    ap.add_argument("--objective", choices=["p99", "p50", "mean", "makespan"], default="p99",
                    help="what the schedule autotuner minimises (uneven workload)")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device-to-device copy of this many GiB three times "
                         "(calibrates the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    dflt = {"paper": (1024, 8, 1000, 1000), "learned": (1024, 16, 64, 16)}.get(args.workload, (256, 32, 256, 256))
    for k, v in zip(("L", "chi", "disorders", "samples"), dflt):
        if getattr(args, k) is None:
            setattr(args, k, v)
    if args.cpu_baseline_child:
        cpu_baseline_child(args.L, args.chi, args.beta, args.samples, args.full_L or args.L,
                           alternate=args.sweeps == "alternating")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the instances are independent and the library runs "
              "on a single MI355X (see the design notes on sharding); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    cpu_proc = None
    if args.workload == "headline" and not args.no_cpu_baseline:
        # the oracle leg runs on the host cores while the GPU forms run
        cpu_proc = start_cpu_baseline(args.L, args.chi, args.beta, alternate=args.sweeps == "alternating")
    import numpy as np
    import torch
    if args.copy_probe > 0:
        n = int(args.copy_probe * (1 << 30))
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: 3 copies of {n} bytes")
        return
    if args.workload == "uneven":
        run_uneven(args)
        return
    if args.workload == "learned":
        run_learned(args)
        return
    if args.workload == "paper":
        run_paper(args)
        return
    if args.workload == "sweep":
        run_sweep(args)
        return
    if args.workload == "rbim":
        run_rbim(args)
        return
    import paper_2509_19006_amd as T
    import workloads
    T.load()

    L, chi, B, N, beta = args.L, args.chi, args.disorders, args.samples, args.beta
    log(f"workload: {B} +-J disorders of {L}x{L}, beta={beta}, chi={chi}, {N} samples each")
    jh_np, jv_np = workloads.batch(L, B, "pmj", 3)
    jh = torch.as_tensor(jh_np).cuda()
    jv = torch.as_tensor(jv_np).cuda()
    seed = 0x5A5A0003

    forms = {}
    names = {"fp32": "plain float32", "bf16x3": "mixed: bf16 matrix-core sampler with split operands",
             "fp16": "float16-stored cache", "bf16": "bfloat16-stored cache"}
    for f in args.forms.split(","):
        log(f"{names[f]} form:")
        forms[f] = run_form(T, torch, T.PRECISIONS[f], jh, jv, L, chi, beta, B, N, args.steps, args.warmup, seed,
                            flags=T.ALTERNATE_SWEEPS if args.sweeps == "alternating" else 0)
    plain = forms["fp32"]

    # the dominant kernel: the cache build (float32 vector ALU, latency bound)
    default_size = (L, chi, B, N) == (256, 32, 256, 256)
    S = plain["jacobi_sweeps_per_site"]
    ex = build_flops_executed(L, chi, B, S)
    dense = build_flops_dense(L, chi, B)
    t_build = plain["build_ms"] * 1e-3
    roof = {"bound": "alu", "kernel": "k_build (cache build, float32 arithmetic)",
            "achieved": ex / t_build / 1e12, "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
            "frac": ex / t_build / PEAK["fp32"],
            "traffic": traffic_for("k_build", "fp32", args.sweeps) if default_size else None,
            "traffic_profile": TRAFFIC_PROFILE,
            "flops_per_launch": ex,
            "per_unit": (f"(2 chi^2 +) (25.3 + 14 S) chi^3 flop per site-row executed by the parity-block "
                         f"kernel, S = {S:.2f} measured Jacobi sweeps per site"),
            "units_per_launch": B * (L - 1) * L,
            "dense_model": {"flops_per_launch": dense, "achieved": dense / t_build / 1e12,
                            "frac": dense / t_build / PEAK["fp32"],
                            "per_unit": "32 chi^2 + 485 chi^3 flop per site-row (dense 2chi blocks, 8 sweeps); "
                                        "not the work the kernel executes"}}
    # the sampler, by form: algorithmic flops and bytes against the roof its
    # intensity selects
    roof_sample = {}
    kinds = {"fp32": (4, PEAK["fp32"], "float32 MFMA"), "bf16x3": (4, PEAK["mfma16"], "bf16 MFMA dense"),
             "fp16": (2, PEAK["mfma16"], "fp16 MFMA dense"), "bf16": (2, PEAK["mfma16"], "bf16 MFMA dense")}
    for name, f in forms.items():
        eb, peak, pname = kinds[name]
        fl, by = sample_flops(L, chi, B, N), sample_bytes(L, chi, B, N, eb)
        t = f["sample_ms"] * 1e-3
        ridge = peak / PEAK["hbm"]
        bound_hbm = fl / by < ridge
        roof_sample[name] = {
            "kernel": "k_sample_mfma", "bound": "hbm" if bound_hbm else "mfma",
            "achieved": (by / t / 1e9) if bound_hbm else (fl / t / 1e12),
            "peak": (PEAK["hbm"] / 1e9) if bound_hbm else (peak / 1e12),
            "unit": "GB/s" if bound_hbm else "TFLOP/s",
            "frac": (by / t / PEAK["hbm"]) if bound_hbm else (fl / t / peak),
            "flops_per_launch": fl, "algorithmic_bytes": by, "intensity_flop_per_byte": fl / by,
            "hbm_frac_of_algorithmic_bytes": by / t / PEAK["hbm"],
            "peak_kind": pname, "traffic": traffic_for("k_sample_mfma", name) if default_size else None}

    cpu = finish_cpu_baseline(cpu_proc) if cpu_proc is not None else None

    line = {
        "metric": METRIC, "value": plain["value"], "unit": "accepted samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": plain["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"TNMC on {L}x{L} open +-J EA lattices, beta={beta}, chi={chi}, {B} disorders x "
                                f"{N} samples: float32 build ({args.sweeps} sweep order"
                                f"{', rows pipelined' if args.sweeps == 'alternating' and chi <= 32 else ''}) and "
                                f"sampler, float64 log-weights and accept, int32 energies; beside it the other "
                                f"precision forms on the same inputs"),
                   "L": L, "chi": chi, "disorders": B, "samples": N, "beta": beta, "form": "plain-fp32",
                   "sweeps": args.sweeps},
        "acceptance": plain["acceptance"],
        "forms": forms,
        "roofline": roof, "roofline_sample": roof_sample, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
