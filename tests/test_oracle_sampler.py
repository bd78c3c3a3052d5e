"""Pins for the oracle row sampler (section 3.3, Eqs. 3-5)."""
import numpy as np
import pytest

import workloads
from oracle import bmps, exact, ising, sampler


def _score_all(L, jh, jv, beta, chi):
    cache, _, lz = bmps.build_cache(beta, jh, jv, chi)
    cf = exact.all_configs(L)
    bits = (cf > 0).astype(np.int64)
    _, lq, _ = sampler.sample(cache, beta, jv, len(cf), forced_bits=bits)
    return cf, lq, lz


@pytest.mark.parametrize("L,fam,beta", [(3, "pmj", 1.0), (3, "gauss", 2.0), (4, "pmj", 0.7),
                                        (4, "gauss", 1.0)])
def test_exact_regime_logq_is_boltzmann(L, fam, beta):
    jh, jv = workloads.instance(L, fam, 21, 0)
    cf, lq, _ = _score_all(L, jh, jv, beta, 2 ** (L // 2))
    want = -beta * ising.energy(cf, jh, jv) - exact.brute_logZ(jh, jv, beta)
    assert np.abs(lq - want).max() < 1e-10 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("chi", [1, 2, 3])
def test_normalised_at_any_chi(chi):
    jh, jv = workloads.instance(4, "gauss", 22, chi)
    _, lq, _ = _score_all(4, jh, jv, 1.5, chi)
    assert abs(np.exp(lq).sum() - 1.0) < 1e-12


@pytest.mark.parametrize("L,chi", [(6, 2), (6, 3), (7, 3)])
def test_truncated_logits_equal_dense_conditionals(L, chi):
    beta = 1.0
    jh, jv = workloads.instance(L, "gauss", 23, chi)
    cache, _, _ = bmps.build_cache(beta, jh, jv, chi)
    psis, _, _ = exact.transfer_vectors(jh, jv, beta, chi=chi)
    s = workloads.random_spins(4, L, 5)
    bits = (s > 0).astype(np.int64)
    _, _, logits = sampler.sample(cache, beta, jv, 4, forced_bits=bits)
    for n in range(4):
        for r in range(L):
            J_up = jv[r - 1] if r > 0 else np.zeros(L)
            u = bits[n, r - 1] if r > 0 else np.zeros(L, dtype=np.int64)
            want = exact.dense_row_logits(psis[r], L, beta, J_up, u, bits[n, r])
            assert np.abs(logits[n, r] - want).max() < 1e-9


def test_z2_symmetry_at_truncated_chi():
    L, chi = 8, 3
    jh, jv = workloads.instance(L, "pmj", 24, 0)
    cache, _, _ = bmps.build_cache(1.0, jh, jv, chi)
    s = workloads.random_spins(6, L, 6)
    _, a, _ = sampler.sample(cache, 1.0, jv, 6, forced_bits=(s > 0).astype(np.int64))
    _, b, _ = sampler.sample(cache, 1.0, jv, 6, forced_bits=(s < 0).astype(np.int64))
    assert np.abs(a - b).max() < 1e-11 * np.abs(a).max()


def test_free_sampling_scores_its_own_draws():
    L, chi = 6, 2
    jh, jv = workloads.instance(L, "gauss", 25, 0)
    cache, _, _ = bmps.build_cache(1.0, jh, jv, chi)
    bits, lq, lg = sampler.sample(cache, 1.0, jv, 16, seed=7, instance=3)
    _, lq2, lg2 = sampler.sample(cache, 1.0, jv, 16, forced_bits=bits)
    assert np.array_equal(lq, lq2) and np.array_equal(lg, lg2)
    b2, _, _ = sampler.sample(cache, 1.0, jv, 8, seed=7, instance=3, sample_offset=8)
    assert np.array_equal(b2, bits[8:])


def test_exact_regime_histogram_is_boltzmann():
    """Drawing with u < p gives the right law: chi-squared on 3x3."""
    from scipy import stats
    L, beta = 3, 0.8
    jh, jv = workloads.instance(L, "gauss", 26, 0)
    cache, _, _ = bmps.build_cache(beta, jh, jv, 2)
    n = 40000
    bits, _, _ = sampler.sample(cache, beta, jv, n, seed=3)
    idx = (bits.reshape(n, -1) * (1 << np.arange(L * L - 1, -1, -1))).sum(axis=1)
    counts = np.bincount(idx, minlength=2 ** (L * L))
    p, _ = exact.brute_probs(jh, jv, beta)
    keep = p * n > 5
    obs = np.append(counts[keep], counts[~keep].sum())
    exp_ = np.append(p[keep] * n, p[~keep].sum() * n)
    assert stats.chisquare(obs, exp_).pvalue > 1e-4
