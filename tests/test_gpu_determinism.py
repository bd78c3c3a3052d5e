"""The cache build and the sampler give the same bits on every run.

A build reads nothing it has not written, and its waves hand data to each
other only through completed barriers: with the workspace filled with zeros,
with 0xFF bytes (NaN in every float type) and reused from the previous call,
ln Z of every instance, the sampled configurations and their log q are
bit-identical (64 x 64 +-J lattices, 16 disorders, chi = 32, so that the
interleaved register Jacobi runs; float64, float32, the mixed form and the
float16 cache; the float forms also with alternating sweeps, where the build
pipelines its rows over two pairs of waves that hand data over through
shared-memory counters).
A race between waves shows as run-to-run differences at rounding level,
which the tolerance-based parity tests cannot see.
"""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,alt", [(0, False), (1, False), (3, False), (4, False), (1, True), (3, True),
                                      (4, True)])
def test_build_and_sample_are_bit_reproducible(tnmc, prec, alt):
    L, B, chi, n = 64, 16, 32, 256
    jh, jv = workloads.batch(L, B, "pmj", 11)
    p = tnmc.Problem(torch.as_tensor(jh).cuda(), torch.as_tensor(jv).cuda(), [L] * B, chi, 1.0,
                     flags=tnmc.ALTERNATE_SWEEPS if alt else 0)
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
        # the build defines its whole statistics record, whatever the
        # workspace held (slot 6 is the sampler's)
        tnmc.tnmc_env_check(env)
        assert (tnmc.tnmc_env_stats(env)[:, 12:] == 0).all()
        outs.append((lz.cpu().numpy(), spins.cpu().numpy(), lq.cpu().numpy()))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
