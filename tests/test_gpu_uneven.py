"""Uneven batches in one launch, and graph capture of the decode steps.

Tolerances as in test_gpu_parity: float32 within 2e-4 * max(1, |value|).
"""
import numpy as np
import pytest

import workloads
from oracle import bmps, sampler

pytestmark = pytest.mark.gpu


def test_uneven_batch_one_launch(tnmc):
    """Mixed L, chi, coupling family and beta in one build launch (float32)."""
    import torch
    import tnmc_gpu as G
    Ls = [8, 12, 16, 20, 8, 12, 16, 20, 6, 10, 14, 18]
    chis = [4, 8, 16, 16, 16, 4, 8, 4, 8, 16, 4, 8]
    fams = ["pmj" if (i // 4) % 2 == 0 else "gauss" for i in range(len(Ls))]
    betas = workloads.betas_uniform(len(Ls), 0.5, 2.0, 90)
    Js = [workloads.instance(L, f, 90, i) for i, (L, f) in enumerate(zip(Ls, fams))]
    G.say(f"uneven batch: L={Ls} chi={chis}")
    jh = torch.as_tensor(np.concatenate([a.ravel() for a, _ in Js])).cuda()
    jv = torch.as_tensor(np.concatenate([b.ravel() for _, b in Js])).cuda()
    p = tnmc.Problem(jh, jv, Ls, chis, betas)
    n = 16
    ws = torch.zeros(tnmc.tnmc_workspace_size(p, tnmc.FP32, n), dtype=torch.uint8, device="cuda")
    logz = torch.zeros(len(Ls), dtype=torch.float64, device="cuda")
    env = tnmc.tnmc_build_env(p, tnmc.FP32, ws, logz)
    draws = []
    for i, (a, b) in enumerate(Js):
        dg = {}
        cache, _, lz = bmps.build_cache(betas[i], a, b, chis[i], dg)
        bits, olq, _ = sampler.sample(cache, betas[i], b, n, seed=5, instance=i)
        draws.append((lz, bits, olq, dg.get("cond", 0.0)))
    words = np.concatenate([G.pack([2 * d[1] - 1]) for d in draws])
    forced = torch.as_tensor(words).cuda()
    spins = torch.zeros_like(forced)
    logq = torch.zeros((len(Ls), n), dtype=torch.float64, device="cuda")
    tnmc.tnmc_sample(env, n, 5, spins, logq, forced_spins=forced)
    torch.cuda.synchronize()
    lz, lq = logz.cpu().numpy(), logq.cpu().numpy()
    st = tnmc.tnmc_env_stats(env)
    for i in range(len(Ls)):
        if draws[i][3] > 1e5:
            continue
        assert abs(lz[i] - draws[i][0]) < 2e-4 * abs(draws[i][0]), i
        assert np.max(np.abs(lq[i] - draws[i][2]) / np.maximum(1, np.abs(draws[i][2]))) < 2e-4, i
    # every instance recorded its build interval and its sampling end
    assert np.all(st[:, 5] > st[:, 4]) and np.all(st[:, 6] >= st[:, 5])


def test_decode_steps_replay_from_a_graph(tnmc):
    """sample -> energy -> accept captured once, replayed three times with
    eager work in between; every replay equals the eager pass."""
    import torch
    import tnmc_gpu as G
    L, chi, B, n = 12, 8, 6, 48
    Js = [workloads.instance(L, "gauss", 91, i) for i in range(B)]
    G.say("graph capture of the decode steps")
    run = G.Run(Js, chi, 1.0, tnmc.FP32, max_samples=n)
    spins = torch.zeros(run.words(n), dtype=torch.int64, device="cuda")
    logq = torch.zeros((B, n), dtype=torch.float64, device="cuda")
    E = torch.zeros((B, n), dtype=torch.float64, device="cuda")
    acc = torch.zeros((B, n), dtype=torch.uint8, device="cuda")
    chain = torch.zeros(B * tnmc.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
    beta = torch.full((B,), 1.0, dtype=torch.float64, device="cuda")

    def decode(stream=None):
        tnmc.tnmc_sample(run.env, n, 77, spins, logq, sample_offset=4096, stream=stream)
        tnmc.tnmc_energy(run.env, n, spins, E, stream=stream)
        tnmc.tnmc_accept(logq, E, beta, chain, 77, 4096, acc, stream=stream)

    decode()
    torch.cuda.synchronize()
    want = [t.clone() for t in (spins, logq, E, acc)]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        chain.zero_()
        with torch.cuda.graph(g, stream=s):
            decode(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for t in (spins, logq, E, acc):
            t.zero_()
        chain.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip((spins, logq, E, acc), want):
            assert torch.equal(a, b), rep
        E.add_(1.0)                   # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec,alt", [(0, False), (1, False), (3, False), (4, False), (1, True), (3, True), (4, True)])
def test_fused_pipeline_equals_separate_calls(tnmc, prec, alt):
    """tnmc_run (build, sampling tiles, energies and the chain in one
    persistent launch) gives bit-identical results to tnmc_build_env +
    tnmc_sample + tnmc_energy + tnmc_accept on an uneven batch; 300 samples
    span two sample tiles, run one after the other in the fused launch.
    With alternating sweeps the float forms build with rows pipelined in
    both."""
    import torch
    import tnmc_gpu as G
    Ls = [6, 12, 20, 9, 16, 24]
    chis = [4, 16, 8, 2, 32 if prec != 0 else 16, 8]
    fams = ["pmj", "gauss", "pmj", "gauss", "gauss", "pmj"]
    betas = workloads.betas_uniform(len(Ls), 0.5, 2.0, 92)
    Js = [workloads.instance(L, f, 92, i) for i, (L, f) in enumerate(zip(Ls, fams))]
    G.say(f"fused pipeline vs separate calls, prec {prec}, alternating {alt}")
    jh = torch.as_tensor(np.concatenate([a.ravel() for a, _ in Js])).cuda()
    jv = torch.as_tensor(np.concatenate([b.ravel() for _, b in Js])).cuda()
    p = tnmc.Problem(jh, jv, Ls, chis, betas, flags=tnmc.ALTERNATE_SWEEPS if alt else 0)
    B, n = len(Ls), 300
    out = []
    for fused in (False, True):
        ws = torch.zeros(tnmc.tnmc_workspace_size(p, prec, n), dtype=torch.uint8, device="cuda")
        spins = torch.zeros(n * p.spin_words_per_sample(), dtype=torch.int64, device="cuda")
        logq = torch.zeros((B, n), dtype=torch.float64, device="cuda")
        E = torch.zeros((B, n), dtype=torch.float64, device="cuda")
        acc = torch.zeros((B, n), dtype=torch.uint8, device="cuda")
        st = torch.zeros((B, n), dtype=torch.int64, device="cuda")
        logz = torch.zeros(B, dtype=torch.float64, device="cuda")
        chain = torch.zeros(B * tnmc.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
        if fused:
            env = tnmc.tnmc_run(p, prec, ws, n, 21, chain, 22, spins, logq, E, acc, st, logz,
                                sample_offset=7, step_offset=7)
        else:
            env = tnmc.tnmc_build_env(p, prec, ws, logz)
            tnmc.tnmc_sample(env, n, 21, spins, logq, sample_offset=7)
            tnmc.tnmc_energy(env, n, spins, E)
            bt = torch.as_tensor(np.asarray(betas, np.float64)).cuda()
            tnmc.tnmc_accept(logq, E, bt, chain, 22, 7, acc, st)
        torch.cuda.synchronize()
        stats = tnmc.tnmc_env_stats(env)
        out.append([t.cpu().numpy() for t in (spins, logq, E, acc, st, logz, chain)] + [stats])
    for a, b in zip(out[0][:7], out[1][:7]):
        assert np.array_equal(a, b)
    # the fused launch records each instance's completion after its build
    st = out[1][7]
    assert np.all(st[:, 6] > st[:, 5]) and np.all(st[:, 5] > st[:, 4])


def test_autotuner_chooses_and_caches(tnmc, tmp_path):
    """The library's tuner times its candidates on a sub-lattice replica,
    returns the best for the objective, appends it to the tuning cache, and
    answers the same batch from the cache without device work."""
    import tnmc_gpu as G
    from paper_2509_19006_amd import autotune
    Ls = [16, 32, 24, 16, 32, 8]
    chis = [16, 32, 64, 8, 16, 32]
    betas = workloads.betas_uniform(len(Ls), 0.5, 2.0, 93)
    Js = [workloads.instance(L, "gauss", 93, i) for i, L in enumerate(Ls)]
    cache = str(tmp_path / "tuning.txt")
    G.say("autotuner: replica timing and tuning cache")
    first = autotune.tune(Js, chis, betas, tnmc.FP32, 16, "p99", 2, cache)
    assert not first["from_cache"]
    assert all(c > 0 for c in first["candidates_s"])
    best = min(range(4), key=lambda k: first["candidates_s"][k])
    assert first["split"] == (best == 3)
    assert first["split"] or first["schedule"] == best
    assert first["objective_s"] == first["candidates_s"][best]
    with open(cache) as f:
        assert len(f.readlines()) == 1
    again = autotune.tune(list(reversed(Js)), list(reversed(chis)), list(reversed(betas)), tnmc.FP32, 16, "p99",
                          2, cache)
    assert again["from_cache"]
    assert (again["schedule"], again["split"]) == (first["schedule"], first["split"])
    # the chosen plan runs the full batch
    res = autotune.run_schedule(Js, chis, betas, tnmc.FP32, 16, first["split"], first["schedule"])
    assert res["trials"] == len(Ls) * 15 and np.all(res["completion_s"] > 0)
