"""Parity of the widest kernels (bond dimensions 33..64: the chi = 64 build
with the accumulated rotation on the second pair of waves, the chi = 64 QR
and sampler) against the float64 oracle, in float32 and in the float16
stored-cache form.

Tolerances: float32 within 2e-4 * max(1, |value|), as in test_gpu_parity;
the float16 stored cache within 2e-3 * max(1, |value|) for log q.
"""
import numpy as np
import pytest

import workloads
from oracle import bmps, exact, ising, sampler

pytestmark = pytest.mark.gpu

TOL = {1: 2e-4, 3: 2e-3}


def rel_err(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(1.0, np.abs(np.asarray(b)))


@pytest.mark.parametrize("prec", [1, 3])
def test_chi64_exact_regime_12x12(tnmc, prec):
    """chi = 64 = 2^(12/2): the boundary MPS is exact, so ln Z equals the
    transfer-vector value and every configuration has log q = -beta E - ln Z.
    Scored on configurations the oracle's sampler draws (typical ones: an
    improbable configuration's conditionals are differences of nearly
    cancelling terms, where float32 keeps few digits)."""
    import tnmc_gpu as G
    L, chi, beta, k = 12, 64, 1.0, 16
    Js = [workloads.instance(L, "gauss", 60, 0), workloads.instance(L, "pmj", 60, 1)]
    G.say(f"chi 64 exact regime 12x12, prec {prec}")
    run = G.Run(Js, chi, beta, prec, max_samples=k)
    spins = []
    for i, (jh, jv) in enumerate(Js):
        cache, _, _ = bmps.build_cache(beta, jh, jv, chi)
        bits, _, _ = sampler.sample(cache, beta, jv, k, seed=600, instance=i)
        spins.append(2 * bits - 1)
    _, lq, _ = run.sample(k, forced=spins)
    for i, (jh, jv) in enumerate(Js):
        _, _, tz = exact.transfer_vectors(jh, jv, beta)
        assert rel_err(run.logz[i], tz) < TOL[1], (i, run.logz[i], tz)
        want = -beta * ising.energy(spins[i], jh, jv) - tz
        print(f"  instance {i}: max relative log q error {rel_err(lq[i], want).max():.2e}")
        assert rel_err(lq[i], want).max() < TOL[prec]


@pytest.mark.parametrize("L,chi,prec", [(20, 64, 1), (16, 48, 1), (20, 64, 3)])
def test_chi_above_32_truncated(tnmc, L, chi, prec):
    """Truncated regime (chi < 2^(L/2)): ln Z and the teacher-forced log q of
    oracle draws (two sample tiles, the second ragged) against the oracle."""
    import tnmc_gpu as G
    beta = 1.0
    Js = [workloads.instance(L, "gauss", 61, 0), workloads.instance(L, "pmj", 61, 1)]
    G.say(f"chi {chi} truncated {L}x{L}, prec {prec}")
    run = G.Run(Js, chi, beta, prec, max_samples=300)
    k, n = 10, 300
    orc, forced = [], []
    for i, (jh, jv) in enumerate(Js):
        dg = {}
        cache, _, lz = bmps.build_cache(beta, jh, jv, chi, dg)
        bits, olq, _ = sampler.sample(cache, beta, jv, k, seed=61, instance=i)
        orc.append((lz, olq, dg.get("cond", 0.0)))
        forced.append(np.tile(2 * bits - 1, (n // k + 1, 1, 1))[:n])
    _, lq, _ = run.sample(n, forced=forced)
    checked = 0
    for i in range(len(Js)):
        lz, olq, cond = orc[i]
        print(f"  instance {i}: truncation conditioning {cond:.1e}, ln Z {run.logz[i]:.8f} vs {lz:.8f}")
        if cond > 1e5:
            continue
        checked += 1
        assert rel_err(run.logz[i], lz) < TOL[1]
        want = np.tile(olq, n // k + 1)[:n]
        print(f"  instance {i}: max relative log q error {rel_err(lq[i], want).max():.2e}")
        assert rel_err(lq[i], want).max() < TOL[prec]
    assert checked >= 1


def test_chi64_in_the_fused_uneven_launch(tnmc):
    """tnmc_run with chi up to 64 in one persistent launch: bit-identical to
    the separate calls, and ln Z of every instance within the float32 bound
    of the oracle."""
    import torch
    import tnmc_gpu as G
    Ls = [12, 20, 8, 16]
    chis = [64, 64, 16, 40]
    fams = ["pmj", "gauss", "gauss", "pmj"]
    betas = workloads.betas_uniform(len(Ls), 0.5, 2.0, 62)
    Js = [workloads.instance(L, f, 62, i) for i, (L, f) in enumerate(zip(Ls, fams))]
    G.say(f"fused launch with chi up to 64: L={Ls} chi={chis}")
    jh = torch.as_tensor(np.concatenate([a.ravel() for a, _ in Js])).cuda()
    jv = torch.as_tensor(np.concatenate([b.ravel() for _, b in Js])).cuda()
    p = tnmc.Problem(jh, jv, Ls, chis, betas)
    B, n, prec = len(Ls), 40, tnmc.FP32
    out = []
    for fused in (False, True):
        ws = torch.zeros(tnmc.tnmc_workspace_size(p, prec, n), dtype=torch.uint8, device="cuda")
        spins = torch.zeros(n * p.spin_words_per_sample(), dtype=torch.int64, device="cuda")
        logq = torch.zeros((B, n), dtype=torch.float64, device="cuda")
        E = torch.zeros((B, n), dtype=torch.float64, device="cuda")
        acc = torch.zeros((B, n), dtype=torch.uint8, device="cuda")
        logz = torch.zeros(B, dtype=torch.float64, device="cuda")
        chain = torch.zeros(B * tnmc.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
        if fused:
            env = tnmc.tnmc_run(p, prec, ws, n, 31, chain, 32, spins, logq, E, acc, None, logz)
        else:
            env = tnmc.tnmc_build_env(p, prec, ws, logz)
            tnmc.tnmc_sample(env, n, 31, spins, logq)
            tnmc.tnmc_energy(p, n, spins, E)
            bt = torch.as_tensor(np.asarray(betas, np.float64)).cuda()
            tnmc.tnmc_accept(logq, E, bt, chain, 32, 0, acc)
        torch.cuda.synchronize()
        tnmc.tnmc_env_check(env)
        out.append([t.cpu().numpy() for t in (spins, logq, E, acc, logz, chain)])
        del env, ws
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    lz = out[0][4]
    for i, (a, b) in enumerate(Js):
        olz = bmps.build_cache(betas[i], a, b, chis[i])[2]
        assert rel_err(lz[i], olz) < TOL[1], (i, lz[i], olz)
