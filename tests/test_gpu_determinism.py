"""The cache build and the sampler give the same bits on every run.

A build reads nothing it has not written, and its waves hand data to each
other only through completed barriers: with the workspace filled with zeros,
with 0xFF bytes (NaN in every float type) and reused from the previous call,
ln Z of every instance, the sampled configurations and their log q are
bit-identical (64 x 64 +-J lattices, 16 disorders, chi = 32, so that the
interleaved register Jacobi runs; float64, float32 and the float16 cache).
A race between waves shows as run-to-run differences at rounding level,
which the tolerance-based parity tests cannot see.
"""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1, 3, 4])
def test_build_and_sample_are_bit_reproducible(tnmc, prec):
    L, B, chi, n = 64, 16, 32, 256
    jh, jv = workloads.batch(L, B, "pmj", 11)
    p = tnmc.Problem(torch.as_tensor(jh).cuda(), torch.as_tensor(jv).cuda(), [L] * B, chi, 1.0)
    ws = torch.empty(tnmc.tnmc_workspace_size(p, prec, n), dtype=torch.uint8, device="cuda")
    outs = []
    for fill in (0, 0xFF, None):
        if fill is not None:
            ws.fill_(fill)
        lz = torch.zeros(B, dtype=torch.float64, device="cuda")
        env = tnmc.tnmc_build_env(p, prec, ws, lz)
        spins = torch.empty(n * p.spin_words_per_sample(), dtype=torch.int64, device="cuda")
        lq = torch.empty((B, n), dtype=torch.float64, device="cuda")
        tnmc.tnmc_sample(env, n, 5, spins, lq)
        torch.cuda.synchronize()
        outs.append((lz.cpu().numpy(), spins.cpu().numpy(), lq.cpu().numpy()))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
