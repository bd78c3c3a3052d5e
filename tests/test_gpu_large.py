"""The largest lattices the library takes (L = 1024, the paper's size) and
the benchmark's full batch, against values that do not come from the GPU:

* closed forms at L = 1024 in one launch: with no vertical couplings every
  row is an open chain and chi = 2 is exact, so ln Z = sum over rows of
  ln(2 prod_c 2 cosh(beta J_c)) and log q(s) = -beta E(s) - ln Z for every
  configuration; at beta = 0 and with every coupling zero, ln Z = L^2 ln 2
  and log q = -L^2 ln 2;
* the paper's instance shape (+-J, 1024 x 1024, beta = 1, chi = 8) and two
  of the benchmark's 256 x 256 disorders (chi = 32): ln Z and the
  teacher-forced log q of configurations drawn by the oracle's own sampler,
  stored by tests/golden/make_golden.py (which calls only the oracle).

Tolerances: float64 within 1e-10 * max(1, |value|) (the closed forms) and
2e-8 relative for the truncated golden cases (below the float64 rounding of
a ~10^6-term sum would not be reachable, and the cut conditioning of the
stored instances is printed); float32 within 2e-4 * max(1, |value|); the
float16 stored cache and the mixed form (bf16 matrix-core products with
split operands) within 5e-4 * max(1, |value|) at full size, with the error
printed per result; the bfloat16 cache's error is printed and bounded
by 3e-2.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {0: 1e-10, 1: 2e-4, 2: 3e-2, 3: 5e-4, 4: 5e-4}


def rel_err(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(1.0, np.abs(np.asarray(b)))


def golden(name):
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_golden import unpack_bits
    with open(os.path.join(HERE, "golden", name)) as f:
        g = json.load(f)
    for inst in g["instances"]:
        inst["spins"] = 2 * unpack_bits(inst["bits"], g["draws"], g["L"]) - 1
    return g


def chain_logz(jh, beta):
    """ln Z of L independent open chains (rows) with couplings jh (L, L-1)."""
    jh = np.asarray(jh, np.float64)
    return float(jh.shape[0] * math.log(2.0) + np.sum(np.log(2.0 * np.cosh(beta * jh))))


def energy(s, jh, jv):
    s = np.asarray(s, np.float64)
    return -(np.sum(jh * s[:, :, :-1] * s[:, :, 1:], axis=(1, 2))
             + np.sum(jv * s[:, :-1, :] * s[:, 1:, :], axis=(1, 2)))


@pytest.mark.parametrize("prec", [0, 1])
def test_closed_forms_at_1024(tnmc, prec):
    import tnmc_gpu as G
    L, n = 1024, 4
    zero_v = np.zeros((L - 1, L), np.float32)
    jh_pmj, _ = workloads.instance(L, "pmj", 70, 0)
    jh_g, _ = workloads.instance(L, "gauss", 70, 1)
    Js = [(jh_pmj, zero_v), (jh_g, zero_v), workloads.instance(L, "gauss", 70, 2),
          (np.zeros((L, L - 1), np.float32), zero_v)]
    betas = [1.0, 0.7, 0.0, 1.5]
    G.say(f"closed forms at L = 1024 (J_v = 0 at chi 2 twice, beta = 0, zero couplings), prec {prec}")
    run = G.Run(Js, 2, betas, prec, max_samples=n)
    tnmc.tnmc_env_check(run.env)
    spins = [workloads.random_spins(n, L, 700 + i) for i in range(4)]
    _, lq, _ = run.sample(n, forced=spins)
    want_z = [chain_logz(jh_pmj, 1.0), chain_logz(jh_g, 0.7), L * L * math.log(2.0), L * L * math.log(2.0)]
    for i in range(4):
        print(f"  instance {i}: ln Z {run.logz[i]:.10f} vs {want_z[i]:.10f}")
        assert rel_err(run.logz[i], want_z[i]) < TOL[prec]
        want = -betas[i] * energy(spins[i], *Js[i]) - want_z[i]
        print(f"  instance {i}: max relative log q error {rel_err(lq[i], want).max():.2e}")
        assert rel_err(lq[i], want).max() < TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_paper_shape_1024_chi8_against_stored_oracle(tnmc, prec):
    import tnmc_gpu as G
    g = golden("paper_1024_chi8.json")
    inst = g["instances"][0]
    L, chi, beta, k = g["L"], g["chi"], g["beta"], g["draws"]
    Js = [workloads.instance(L, g["family"], g["config_id"], inst["index"])]
    G.say(f"paper shape 1024x1024 chi {chi}, prec {prec} (cut conditioning {inst['cond']:.1e})")
    run = G.Run(Js, chi, beta, prec, max_samples=2 * k)
    tnmc.tnmc_env_check(run.env)
    forced = [np.concatenate([inst["spins"], -inst["spins"]])]
    _, lq, _ = run.sample(2 * k, forced=forced)
    tol = 2e-8 if prec == 0 else TOL[1]
    print(f"  ln Z {run.logz[0]:.8f} vs {inst['logz']:.8f}; log q {lq[0].tolist()} vs {inst['logq']}")
    assert rel_err(run.logz[0], inst["logz"]) < tol
    want = np.concatenate([inst["logq"], inst["logq"]])          # Z2 partners score the same
    assert rel_err(lq[0], want).max() < tol


def test_full_size_batch_forms_against_stored_oracle(tnmc):
    """The benchmark's launch configuration (256 +-J disorders of 256 x 256,
    chi 32, 256 samples in one build and one sampling launch) in float32 and
    in the float16 and bfloat16 stored-cache forms: the two stored
    instances' ln Z and teacher-forced log q against the oracle; every
    instance's draws score the same as their spin flips (Z2)."""
    import torch
    import tnmc_gpu as G
    g = golden("fullsize_256_chi32.json")
    L, chi, beta, k = g["L"], g["chi"], g["beta"], g["draws"]
    B, N = 256, 256
    jh, jv = workloads.batch(L, B, g["family"], g["config_id"])
    Js = [(jh[i], jv[i]) for i in range(B)]
    for prec in (tnmc.FP32, tnmc.MIXED_BF16X3, tnmc.MIXED_FP16, tnmc.MIXED_BF16):
        G.say(f"full size: {B} x {L}x{L}, chi {chi}, {N} samples, prec {prec}")
        run = G.Run(Js, chi, beta, prec, max_samples=N)
        tnmc.tnmc_env_check(run.env)
        sp, lq, _ = run.sample(N, seed=0x5A5A0003)
        assert np.all(np.isfinite(run.logz)) and np.all(np.isfinite(lq)) and np.all(lq < 0)
        m = 8
        _, lq_f, _ = run.sample(m, forced=[-s[:m] for s in sp])
        z2 = rel_err(lq_f, lq[:, :m]).max()
        print(f"  Z2: max relative log q difference {z2:.2e}")
        assert z2 < TOL[1]
        forced = [np.zeros((k, L, L), np.int8) + 1 for _ in range(B)]
        for inst in g["instances"]:
            forced[inst["index"]] = inst["spins"]
        _, lq_o, _ = run.sample(k, forced=forced)
        for inst in g["instances"]:
            i = inst["index"]
            ez = rel_err(run.logz[i], inst["logz"])
            eq = rel_err(lq_o[i], inst["logq"]).max()
            print(f"  instance {i}: ln Z relative error {ez:.2e}, log q relative error {eq:.2e} "
                  f"(|log q| ~ {abs(inst['logq'][0]):.0f}, cut conditioning {inst['cond']:.1e})")
            assert ez < TOL[1]                      # ln Z comes from the float32 build in every form
            assert eq < TOL[prec]
        del run
        torch.cuda.empty_cache()


def test_full_size_pipelined_build_against_stored_oracle(tnmc):
    """The benchmark's launch configuration with the alternating sweep order
    (256 +-J disorders of 256 x 256, chi 32, 256 samples; the float builds
    then pipeline their rows) in float32, the mixed form and the float16
    cache: the two stored instances' ln Z and teacher-forced log q against
    the oracle's alternating compression; no hand-over lost."""
    import torch
    import tnmc_gpu as G
    g = golden("fullsize_256_chi32_alt.json")
    assert g["alternate"]
    L, chi, beta, k = g["L"], g["chi"], g["beta"], g["draws"]
    B, N = 256, 256
    jh, jv = workloads.batch(L, B, g["family"], g["config_id"])
    Js = [(jh[i], jv[i]) for i in range(B)]
    for prec in (tnmc.FP32, tnmc.MIXED_BF16X3, tnmc.MIXED_FP16):
        G.say(f"full size, alternating sweeps: {B} x {L}x{L}, chi {chi}, prec {prec}")
        run = G.Run(Js, chi, beta, prec, max_samples=N, flags=tnmc.ALTERNATE_SWEEPS)
        tnmc.tnmc_env_check(run.env)
        assert (run.stats()[:, tnmc.STAT_PIPE_ERROR] == 0).all()
        forced = [np.zeros((k, L, L), np.int8) + 1 for _ in range(B)]
        for inst in g["instances"]:
            forced[inst["index"]] = inst["spins"]
        _, lq_o, _ = run.sample(k, forced=forced)
        for inst in g["instances"]:
            i = inst["index"]
            ez = rel_err(run.logz[i], inst["logz"])
            eq = rel_err(lq_o[i], inst["logq"]).max()
            print(f"  instance {i}: ln Z relative error {ez:.2e}, log q relative error {eq:.2e} "
                  f"(cut conditioning {inst['cond']:.1e})")
            assert ez < TOL[1]
            assert eq < TOL[prec]
        del run
        torch.cuda.empty_cache()
