#!/usr/bin/env python3
"""Throughput of the batched TNMC hot path on one MI355X.

One step = the whole path over one batch of synthetic disorders: boundary-MPS
cache build (tnmc_build_env), sampling (tnmc_sample), exact energies
(tnmc_energy) and the Metropolis independence step (tnmc_accept), all on one
stream with the couplings already resident in HBM.  Workload (default): the
mixed-precision configuration -- 256 x 256 open-boundary +-J Edwards-Anderson
lattices, beta = 1, chi = 32, 256 disorders x 256 samples; the same inputs are
also run through the plain float32 path.  The Markov chains continue across
steps; accepted samples are accepted Metropolis trials.

Prints one JSON line (rank 0) with the headline value (mixed form), the plain
float32 comparison, a roofline entry for the dominant kernel (the cache
build) and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

METRIC = "accepted samples/s at L=256 chi=32 + acceptance rate, learned/mixed vs plain"
PEAK = {"fp32": 157.3e12, "fp64": 78.6e12}          # MI355X vector peaks, flop/s

# HBM traffic of one cache-build launch at the default workload, from two
# rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE) scaled by the same counters
# read for a plain copy of known size; valid only for the kernel source it
# was measured on (sha256 over the files below), reported as null otherwise.
TRAFFIC_SOURCES = ["paper_2509_19006_amd/csrc/build.hip", "paper_2509_19006_amd/csrc/build_device.hpp",
                   "paper_2509_19006_amd/csrc/device.hpp"]
TRAFFIC = {"sha256": "e934049df3328d5f7e2e9a1202f3601e92499ed3f98c4e996ba97a901a385582",
           "bytes": 870260078330,
           "profile": "profiles/k_build_k_sample_c3_fp16_hbm_traffic.txt"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_for_current_kernel():
    import hashlib
    if TRAFFIC is None:
        return None
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC["bytes"] if h.hexdigest() == TRAFFIC["sha256"] else None


def build_flops_model(L, chi, B):
    """Algorithmic flops of one cache build: per site of every row above the
    bottom one, 32 chi^2 + (101 + 48 S) chi^3 with S = 8 Jacobi sweeps (the
    dense boundary-MPS cost model: MPO apply, QR sweep, SVD sweep)."""
    per_site = 32 * chi ** 2 + (101 + 48 * 8) * chi ** 3
    return B * (L - 1) * L * per_site


def run_form(T, torch, prec, jh, jv, L, chi, beta, B, N, steps, warmup, seed):
    problem = T.Problem(jh, jv, [L] * B, chi, beta)
    nbytes = T.tnmc_workspace_size(problem, prec, N)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    words = N * problem.spin_words_per_sample()
    spins = torch.empty(words, dtype=torch.int64, device="cuda")
    logq = torch.empty((B, N), dtype=torch.float64, device="cuda")
    E = torch.empty((B, N), dtype=torch.float64, device="cuda")
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
        T.tnmc_energy(env, N, spins, E)
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
    out = dict(value=n_acc / wall, acceptance=n_acc / max(1, n_tr), accepted=n_acc, trials=n_tr,
               wall_s=wall, ms_per_step=1e3 * wall / steps,
               build_ms=phase[0], sample_ms=phase[1], energy_ms=phase[2], accept_ms=phase[3],
               jacobi_sweeps_per_site=float(stats[:, 0].mean()) / ((L - 1) * L),
               logz_mean=float(logz.mean().item()))
    del envs, ws
    torch.cuda.empty_cache()
    return out


def cpu_baseline(L, chi, beta, N, acceptance, jh, jv, build_rows=36, sample_rows=3, n_sample=8):
    """The oracle, timed on a bounded sample of one instance of the workload:
    `build_rows` bulk rows of the cache build (after the bonds have reached
    chi) and `sample_rows` rows of sampling for `n_sample` samples, scaled to
    a whole instance (L-1 rows built, N samples of L rows)."""
    import numpy as np
    from oracle import bmps, sampler
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = len(os.sched_getaffinity(0))
    jh = jh.astype(np.float64)
    jv = jv.astype(np.float64)
    mps, _ = bmps.bottom_row_mps(beta, jh)
    row = L - 2
    for _ in range(int(math.log2(chi)) + 2):                 # bonds grow to chi
        mps = bmps.multiply(bmps.row_mpo(beta, jh, jv, row), mps)
        _, mps = bmps.compress(mps, chi)
        row -= 1
    t0 = time.perf_counter()
    for _ in range(build_rows):
        mps = bmps.multiply(bmps.row_mpo(beta, jh, jv, row), mps)
        _, mps = bmps.compress(mps, chi)
        row -= 1
    t_row = (time.perf_counter() - t0) / build_rows
    rng = np.random.default_rng(0)
    u = rng.integers(0, 2, (n_sample, L))
    t0 = time.perf_counter()
    for _ in range(sample_rows):
        sampler.sample_row(mps, beta, jv[row], u, n_sample, uniforms=rng.random((n_sample, L)))
    t_srow = (time.perf_counter() - t0) / (sample_rows * n_sample)
    per_instance = (L - 1) * t_row + N * L * t_srow
    return {"value": acceptance * N / per_instance, "unit": "accepted samples/s", "cores": int(cores),
            "kind": "oracle",
            "sample": (f"one {L}x{L} chi={chi} instance: {build_rows} bulk rows of the float64 cache "
                       f"build ({t_row:.3f} s/row) and {sample_rows} rows x {n_sample} samples of "
                       f"sampling ({t_srow * 1e3:.2f} ms per sample-row), scaled to {L - 1} rows and "
                       f"{N} samples; acceptance taken from the float32 GPU run")}


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
    log(f"uneven batch: {len(spec)} instances, {N} samples each; tuning the schedule on a 1/4-scale replica "
        f"(objective {args.objective})")
    name, mode, order, table = autotune.tune(lambda L, fam, i: workloads.instance(L, fam, 40, i), spec, T.FP32,
                                             N, objective=args.objective, scale=4)
    for k, (v, r) in table.items():
        c = r["completion_s"]
        log(f"  {k}: {args.objective} {v:.3f} s, wall {r['wall_s']:.3f} s, p50 {np.percentile(c, 50):.3f} s, "
            f"p99 {np.percentile(c, 99):.3f} s")
    log(f"chosen: {name}; full batch ...")
    Js = [workloads.instance(L, fam, 4, i) for i, (L, fam, _, _) in enumerate(spec)]
    res = autotune.run_schedule(Js, [c for _, _, c, _ in spec], [b for _, _, _, b in spec], T.FP32, N, mode, order)
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
        "tuner_replica": {k: {"objective": v, "wall_s": r["wall_s"],
                              "p50_s": float(np.percentile(r["completion_s"], 50)),
                              "p99_s": float(np.percentile(r["completion_s"], 99))}
                          for k, (v, r) in table.items()},
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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--chi", type=int, default=32)
    ap.add_argument("--disorders", type=int, default=256)
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--beta", type=float, default=1.0)
    ap.add_argument("--mixed", choices=["bf16", "fp16"], default="fp16")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain float32 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["mixed", "uneven", "learned"], default="mixed",
                    help="mixed: the headline 256x256 batch (default); uneven: the 512-instance mix in one "
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
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the instances are independent and this build runs "
              "on a single MI355X; use --gpus 1", file=sys.stderr)
        sys.exit(2)

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
    import paper_2509_19006_amd as T
    import workloads
    T.load()

    L, chi, B, N, beta = args.L, args.chi, args.disorders, args.samples, args.beta
    log(f"workload: {B} +-J disorders of {L}x{L}, beta={beta}, chi={chi}, {N} samples each")
    jh_np, jv_np = workloads.batch(L, B, "pmj", 3)
    jh = torch.as_tensor(jh_np).cuda()
    jv = torch.as_tensor(jv_np).cuda()
    seed = 0x5A5A0003

    mixed_prec = T.MIXED_BF16 if args.mixed == "bf16" else T.MIXED_FP16
    log(f"mixed form ({args.mixed} cache, float32 build):")
    mixed = run_form(T, torch, mixed_prec, jh, jv, L, chi, beta, B, N, args.steps, args.warmup, seed)
    plain = None
    if not args.no_plain:
        log("plain float32 form:")
        plain = run_form(T, torch, T.FP32, jh, jv, L, chi, beta, B, N, args.steps, args.warmup, seed)

    flops = build_flops_model(L, chi, B)
    achieved = flops / (mixed["build_ms"] * 1e-3)
    roof = {"bound": "alu", "kernel": "k_build (cache build, float32 arithmetic)",
            "achieved": achieved / 1e12, "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK["fp32"],
            "traffic": (traffic_for_current_kernel()
                        if (L, chi, B, args.mixed) == (256, 32, 256, "fp16") else None),
            "flops_per_launch": flops,
            "per_unit": "32 chi^2 + 485 chi^3 flop per site-row (dense cost model, 8 sweeps)",
            "units_per_launch": B * (L - 1) * L}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        acc_ref = (plain or mixed)["acceptance"]
        cpu = cpu_baseline(L, chi, beta, N, acc_ref, jh_np[0], jv_np[0])

    line = {
        "metric": METRIC, "value": mixed["value"], "unit": "accepted samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"mixed-precision TNMC: {L}x{L} open +-J EA lattices, beta={beta}, "
                                f"chi={chi}, {B} disorders x {N} samples, {args.mixed} cache, float32 "
                                "build, float64 log-weights and accept"),
                   "L": L, "chi": chi, "disorders": B, "samples": N, "beta": beta,
                   "form": f"mixed-{args.mixed}"},
        "acceptance": mixed["acceptance"],
        "mixed": mixed, "plain_fp32": plain,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
