"""Pins for the exact references themselves (brute force, transfer vectors,
the mean energy by differentiation) and for the truncation diagnostic."""
import math

import numpy as np
import pytest

import workloads
from oracle import bmps, exact


@pytest.mark.parametrize("L,fam", [(3, "pmj"), (3, "gauss"), (4, "pmj"), (4, "gauss")])
@pytest.mark.parametrize("beta", [0.4, 1.0, 1.7])
def test_mean_energy_equals_brute_force_average(L, fam, beta):
    """<E> = sum_s P(s) E(s) over all 2**(L*L) configurations (Eq. 2)."""
    jh, jv = workloads.instance(L, fam, 41, L)
    p, E = exact.brute_probs(jh, jv, beta)
    want = float((p * E).sum())
    got = exact.transfer_mean_energy(jh, jv, beta)
    assert abs(got - want) < 1e-11 * max(1.0, abs(want))


@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_mean_energy_is_minus_dlnZ_dbeta(beta):
    """<E> = -d ln Z / d beta, against a central difference of the transfer
    vector's ln Z at L = 6 (step 1e-4: truncation error ~ h**2 * ln Z''')."""
    jh, jv = workloads.instance(6, "gauss", 42, 0)
    h = 1e-4
    zp = exact.transfer_vectors(jh, jv, beta + h)[2]
    zm = exact.transfer_vectors(jh, jv, beta - h)[2]
    fd = -(zp - zm) / (2 * h)
    got = exact.transfer_mean_energy(jh, jv, beta)
    assert abs(got - fd) < 1e-6 * max(1.0, abs(fd))


def test_mean_energy_limits():
    """beta = 0: every configuration equally likely, <E> = 0; a ferromagnet
    at large beta sits in its ground state, <E> -> -(number of bonds)."""
    L = 5
    jh = np.ones((L, L - 1), np.float32)
    jv = np.ones((L - 1, L), np.float32)
    assert abs(exact.transfer_mean_energy(jh, jv, 0.0)) < 1e-12
    nb = 2 * L * (L - 1)
    assert abs(exact.transfer_mean_energy(jh, jv, 12.0) + nb) < 1e-6


def _mps_from_dense(psi, L):
    """Exact MPS of a dense 2**L vector by successive SVDs (no truncation)."""
    out = []
    rest = psi.reshape(1, -1)
    for c in range(L - 1):
        Dl = rest.shape[0]
        M = rest.reshape(Dl * 2, -1)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        k = int((S > 1e-14 * S[0]).sum())
        out.append(U[:, :k].reshape(Dl, 2, k))
        rest = S[:k, None] * Vt[:k]
    out.append(rest.reshape(rest.shape[0], 2, 1))
    return out


@pytest.mark.parametrize("sig,keep", [((1.0, 0.5, 0.3, 0.29), 3), ((1.0, 0.6, 0.59, 0.1), 2),
                                      ((1.0, 0.2, 0.1, 0.05), 1)])
def test_compress_cut_conditioning_on_known_spectrum(sig, keep):
    """A 4-site state whose middle cut has the prescribed Schmidt values;
    with chi = keep only that cut discards anything (the outer cuts have
    rank <= 2 <= chi unless keep = 1), and the diagnostic must equal
    sigma_k / (sigma_k - sigma_{k+1}) for that cut."""
    rng = np.random.default_rng(7)
    U, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    V, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    M = U @ np.diag(sig) @ V.T
    mps = _mps_from_dense(M.reshape(-1), 4)
    diag = {}
    bmps.compress(mps, keep, diag)
    s = np.asarray(sig) / np.linalg.norm(sig)
    want = s[keep - 1] / (s[keep - 1] - s[keep])
    if keep >= 2:
        assert abs(diag["cond"] - want) < 1e-9 * want
    else:
        # chi = 1 also truncates the outer cuts (rank 2): the diagnostic is
        # the worst cut, at least the middle one's
        assert diag["cond"] >= want * (1 - 1e-9)


def test_compress_reports_exact_tie_as_infinite():
    rng = np.random.default_rng(8)
    U, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    V, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    M = U @ np.diag([1.0, 0.5, 0.5, 0.1]) @ V.T
    diag = {}
    bmps.compress(_mps_from_dense(M.reshape(-1), 4), 2, diag)
    assert diag["cond"] > 1e12


def test_compress_without_discarding_reports_nothing():
    rng = np.random.default_rng(9)
    psi = rng.normal(size=2 ** 5)
    diag = {}
    ln, out = bmps.compress(_mps_from_dense(psi, 5), 4, diag)
    assert "cond" not in diag
    assert abs(ln - math.log(np.linalg.norm(psi))) < 1e-12
    v = bmps.mps_to_dense(out)
    assert np.abs(np.abs(v @ psi) / np.linalg.norm(psi) - 1.0) < 1e-12
