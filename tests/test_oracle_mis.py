"""Pins for the oracle Metropolis independence chain (Eq. 10)."""
import numpy as np

import workloads
from oracle import bmps, exact, ising, mis, sampler


def _proposals(L, fam, beta, chi, n, seed):
    jh, jv = workloads.instance(L, fam, 31, seed)
    cache, _, _ = bmps.build_cache(beta, jh, jv, chi)
    bits, lq, _ = sampler.sample(cache, beta, jv, n, seed=seed)
    E = ising.energy(2 * bits - 1, jh, jv)
    return jh, jv, bits, lq, E


def test_exact_regime_accepts_everything():
    jh, jv, bits, lq, E = _proposals(6, "pmj", 1.0, 8, 64, 1)
    ch = mis.Chain()
    acc, idx = mis.accept(lq, E, 1.0, ch, seed=5, instance=0, step_offset=0)
    assert ch.n_trials == 63 and ch.n_acc == 63 and acc.all()
    assert np.array_equal(idx, np.arange(64))


def test_chain_split_equals_uninterrupted():
    _, _, _, lq, E = _proposals(5, "gauss", 1.0, 2, 40, 2)
    a = mis.Chain()
    acc_a, idx_a = mis.accept(lq, E, 1.0, a, 9, 4, 0)
    b = mis.Chain()
    acc_1, idx_1 = mis.accept(lq[:17], E[:17], 1.0, b, 9, 4, 0)
    acc_2, idx_2 = mis.accept(lq[17:], E[17:], 1.0, b, 9, 4, 17)
    assert np.array_equal(acc_a, np.concatenate([acc_1, acc_2]))
    assert np.array_equal(idx_a, np.concatenate([idx_1, idx_2]))
    assert (a.n_acc, a.n_trials) == (b.n_acc, b.n_trials)


def test_truncated_chain_is_unbiased():
    """At chi = 1 on 3x3 the proposal is visibly wrong, the chain is not."""
    from scipy import stats
    L, beta, n = 3, 1.2, 30000
    jh, jv, bits, lq, E = _proposals(L, "gauss", beta, 1, n, 3)
    ch = mis.Chain()
    _, idx = mis.accept(lq, E, beta, ch, 11, 0, 0)
    code = (bits.reshape(n, -1) * (1 << np.arange(L * L - 1, -1, -1))).sum(axis=1)
    p, _ = exact.brute_probs(jh, jv, beta)

    def pval(c):
        counts = np.bincount(c, minlength=2 ** (L * L))
        keep = p * len(c) > 5
        obs = np.append(counts[keep], counts[~keep].sum())
        ex = np.append(p[keep] * len(c), p[~keep].sum() * len(c))
        return stats.chisquare(obs, ex).pvalue

    assert pval(code) < 1e-6                      # raw proposals are biased
    # the chain is correlated (integrated autocorrelation ~12 proposals here):
    # thin it well past that before a test that assumes independence
    assert pval(code[idx[1000::30]]) > 1e-4
    # and its mean energy agrees with the exact one within batch-means errors
    e_chain = E[idx[1000:]]
    nb = 20
    means = e_chain[: len(e_chain) // nb * nb].reshape(nb, -1).mean(axis=1)
    err = means.std(ddof=1) / np.sqrt(nb)
    e_exact = (p * exact.brute_energies(jh.astype(float), jv.astype(float))).sum()
    assert abs(e_chain.mean() - e_exact) < 4 * err
    assert abs(E.mean() - e_exact) > 20 * err
    assert 0.1 < ch.n_acc / ch.n_trials < 1.0
