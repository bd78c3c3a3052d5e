"""The corrected chain is unbiased, and float32 agrees with float64.

(1) 16x16 Gaussian couplings, chi = 2 (truncated far below the exact bond
dimension 256, so that the correction rejects a sizeable share), beta in
{0.5, 1, 2}: the mean energy of the Metropolis-corrected chain matches the
exact mean energy from the transfer vector within its statistical error
(batch means over 16 batches of 2048 trials; |z| < 4.5), for the float64 and
the float32 paths.  This pins the whole path (build, sampler, energy,
accept) against exact physics rather than against the oracle's own
arithmetic.

(2) 64x64 Gaussian couplings, chi = 32, beta in {0.5, 1, 2}, 100 disorders x
100 samples in one batched launch, float32 against float64: acceptance rates
are printed; the disorder-averaged chain energy per spin of the two paths
agrees within 4 standard errors of their paired difference.
"""
import numpy as np
import pytest

import workloads
from oracle import exact

pytestmark = pytest.mark.gpu


def chain_energies(G, lq, E, beta, seed):
    """Energy of the chain state after every trial (proposal 0 starts it)."""
    B, n = lq.shape
    _, st, _ = G.gpu_accept(lq, E, np.full(B, beta), seed, 0)
    return np.take_along_axis(E, st[:, 1:], axis=1), st


def batch_means(x, nb=16):
    m = len(x) // nb
    b = x[: m * nb].reshape(nb, m).mean(axis=1)
    return b.mean(), b.std(ddof=1) / np.sqrt(nb)


@pytest.mark.parametrize("prec", [0, 1])
def test_chain_mean_energy_is_exact_at_16x16(tnmc, prec):
    import tnmc_gpu as G
    L, chi, B, n = 16, 2, 3, 32768
    for beta in (0.5, 1.0, 2.0):
        Js = [workloads.instance(L, "gauss", 80, i) for i in range(B)]
        G.say(f"C2 exactness: 16x16 chi {chi} beta {beta} prec {prec}, {B} x {n} samples")
        run = G.Run(Js, chi, beta, prec, max_samples=n)
        sp, lq, _ = run.sample(n, seed=0x5A5A0002)
        E = run.energy(sp)
        Ec, st = chain_energies(G, lq, E, beta, 0x5A5A0002)
        acc = np.mean(st[:, 1:] != st[:, :-1])
        for i, (jh, jv) in enumerate(Js):
            ex = exact.transfer_mean_energy(jh, jv, beta)
            m, se = batch_means(Ec[i])
            z = (m - ex) / se
            print(f"  inst {i}: <E> chain {m:.3f} +- {se:.3f}, exact {ex:.3f}, z {z:+.2f}, acceptance {acc:.3f}")
            assert abs(z) < 4.5, (beta, i, m, se, ex)


def test_float32_matches_float64_at_64x64(tnmc):
    import tnmc_gpu as G
    L, chi, B, n = 64, 32, 100, 100
    for beta in (0.5, 1.0, 2.0):
        Js = [workloads.instance(L, "gauss", 2, i) for i in range(B)]
        per = {}
        for prec in (0, 1):
            G.say(f"C2: 64x64 chi {chi} beta {beta} prec {prec}, {B} x {n}")
            run = G.Run(Js, chi, beta, prec, max_samples=n)
            sp, lq, _ = run.sample(n, seed=0x5A5A0002)
            E = run.energy(sp)
            Ec, st = chain_energies(G, lq, E, beta, 0x5A5A0002)
            acc = np.mean(st[:, 1:] != st[:, :-1], axis=1)
            per[prec] = (Ec.mean(axis=1) / L ** 2, acc)
            del run
        d = per[1][0] - per[0][0]
        se = d.std(ddof=1) / np.sqrt(B)
        e64, e32 = per[0][0].mean(), per[1][0].mean()
        s64 = per[0][0].std(ddof=1) / np.sqrt(B)
        print(f"  beta {beta}: <E>/N float64 {e64:.5f} +- {s64:.5f}, float32 {e32:.5f}, "
              f"difference {d.mean():+.2e} +- {se:.1e}; acceptance float64 {per[0][1].mean():.3f}, "
              f"float32 {per[1][1].mean():.3f}")
        assert abs(d.mean()) <= 4 * se + 1e-12
        assert abs(per[0][1].mean() - per[1][1].mean()) < 0.05
