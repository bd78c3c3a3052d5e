"""Parity at the benchmark's full size, in the launch configuration bench.py
times: 256 +-J disorders of 256x256, beta = 1, chi = 32, 256 samples, one
build launch and one sampling launch over the whole batch (float32).

The float64 oracle builds two of the instances (about half a minute each on
the host) and scores a few of the GPU's own draws (teacher forcing): ln Z
and those log q agree within the float32 bound 2e-4 * max(1, |value|).  For
every instance a property that holds at any size is checked: the spin-flipped
draws score the same log q (Z2 symmetry of the proposal).
"""
import numpy as np
import pytest

import workloads
from oracle import bmps, sampler

pytestmark = pytest.mark.gpu

L, CHI, B, N, BETA = 256, 32, 256, 256, 1.0


def test_full_size_batch_against_oracle(tnmc):
    import torch
    import tnmc_gpu as G
    jh, jv = workloads.batch(L, B, "pmj", 3)
    G.say(f"full size: {B} x {L}x{L}, chi {CHI}, {N} samples, float32 (build ~10 s)")
    Js = [(jh[i], jv[i]) for i in range(B)]
    run = G.Run(Js, CHI, BETA, tnmc.FP32, max_samples=N)
    sp, lq, _ = run.sample(N, seed=0x5A5A0003)
    lz = run.logz
    assert np.all(np.isfinite(lz)) and np.all(np.isfinite(lq)) and np.all(lq < 0)
    G.say("  spin-flipped draws, all instances")
    k = 8
    _, lq_f, _ = run.sample(k, forced=[-s[:k] for s in sp])
    rel = np.abs(lq_f - lq[:, :k]) / np.maximum(1.0, np.abs(lq[:, :k]))
    print(f"  Z2: max relative log q difference {rel.max():.2e}")
    assert rel.max() < 2e-4
    for i in (0, 1):
        G.say(f"  oracle build of instance {i} (float64, host)")
        dg = {}
        cache, _, olz = bmps.build_cache(BETA, jh[i], jv[i], CHI, dg)
        print(f"  instance {i}: ln Z gpu {lz[i]:.6f} oracle {olz:.6f}, truncation conditioning {dg.get('cond', 0):.1e}")
        assert abs(lz[i] - olz) < 2e-4 * abs(olz)
        m = 3
        bits = (sp[i][:m] > 0).astype(np.int64)
        _, olq, _ = sampler.sample(cache, BETA, jv[i], m, forced_bits=bits)
        r = np.abs(lq[i][:m] - olq) / np.maximum(1.0, np.abs(olq))
        print(f"  instance {i}: teacher-forced log q max relative error {r.max():.2e}")
        assert r.max() < 2e-4
