"""Exact references for small lattices (oracle side, float64).

Test infrastructure only: nothing in the product path imports this module.
These share no code with the boundary-MPS oracle (bmps.py / sampler.py); they
are what pins it:

* brute-force enumeration of the Boltzmann law of Eq. (2) (N = L*L <= 16);
* the dense transfer vector psi_r(s_row) of length 2**L (L <= 16), built row
  by row from the bottom as in Eq. (6) with no approximation; with a chi it
  applies the same sequential right-to-left Schmidt truncation to the dense
  vector, which is what the MPS compress computes when its left part is
  canonical (section 2.2, Fig. 2);
* conditionals of a row computed directly from a dense row vector;
* the exact mean energy as -d ln Z / d beta, carried through the transfer
  vector with its beta-derivative.

Pins (tests/test_oracle_exact.py, tests/test_oracle_bmps.py): the transfer
vector's ln Z equals brute-force enumeration; the mean energy equals the
brute-force Boltzmann average on 3x3 and 4x4, a central difference of ln Z
in beta at L = 6, and the beta = 0 and ground-state limits.

Dense vectors index the row's spins with column 0 as the most significant bit
and bit value 1 meaning spin +1.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def all_configs(L: int) -> np.ndarray:
    """All 2**(L*L) configurations, shape (2**N, L, L), values -1/+1, site
    (0,0) the most significant bit."""
    N = L * L
    idx = np.arange(2 ** N, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(N - 1, -1, -1)[None, :]) & 1
    return (2 * bits - 1).reshape(-1, L, L).astype(np.int8)


def brute_energies(J_h, J_v):
    """Energies of every configuration, computed bond by bond from the
    per-site (left, up, right, down) table and halved (every bond is seen
    from both ends) -- deliberately a different route from ising.energy."""
    L = J_h.shape[0]
    s = all_configs(L).astype(np.float64)
    E = np.zeros(s.shape[0])
    for r in range(L):
        for c in range(L):
            nb = 0.0
            if c > 0:
                nb = nb + J_h[r, c - 1] * s[:, r, c - 1]
            if c < L - 1:
                nb = nb + J_h[r, c] * s[:, r, c + 1]
            if r > 0:
                nb = nb + J_v[r - 1, c] * s[:, r - 1, c]
            if r < L - 1:
                nb = nb + J_v[r, c] * s[:, r + 1, c]
            E -= 0.5 * s[:, r, c] * nb
    return E


def brute_logZ(J_h, J_v, beta):
    E = brute_energies(np.asarray(J_h, np.float64), np.asarray(J_v, np.float64))
    x = -beta * E
    m = x.max()
    return float(m + math.log(np.exp(x - m).sum()))


def brute_probs(J_h, J_v, beta):
    E = brute_energies(np.asarray(J_h, np.float64), np.asarray(J_v, np.float64))
    x = -beta * E
    w = np.exp(x - x.max())
    return w / w.sum(), E


def _row_spins(L):
    idx = np.arange(2 ** L, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(L - 1, -1, -1)[None, :]) & 1
    return 2.0 * bits - 1.0                                    # (2**L, L)


def _apply_site_matrices(psi, mats):
    """psi (2**L,) -> (tensor product of 2x2 mats) psi, mats[c] on column c."""
    L = len(mats)
    t = psi.reshape((2,) * L)
    for c, M in enumerate(mats):
        t = np.moveaxis(np.tensordot(M, t, axes=(1, c)), 0, c)
    return t.reshape(-1)


def _truncate_dense(psi, L, chi, mirrored=False):
    """Sequential Schmidt truncation, bond (L-2|L-1) first, then leftwards;
    mirrored: bond (0|1) first, then rightwards."""
    if mirrored:
        psi = psi.reshape((2,) * L).transpose(tuple(range(L - 1, -1, -1))).reshape(-1)
    for c in range(L - 1, 0, -1):
        M = psi.reshape(2 ** c, 2 ** (L - c))
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        k = min(chi, S.shape[0])
        psi = ((U[:, :k] * S[:k]) @ Vt[:k]).reshape(-1)
    if mirrored:
        psi = psi.reshape((2,) * L).transpose(tuple(range(L - 1, -1, -1))).reshape(-1)
    return psi


def transfer_vectors(J_h, J_v, beta, chi=None, alternate=False):
    """Row vectors psi_r (normalised) and the log-scales taken out.

    psi_r(s) is proportional to sum over rows > r of exp(-beta E(rows >= r));
    with chi, every row above the bottom one is truncated after the vertical
    and horizontal weights are applied.  Returns (list of psi_r, logscales,
    logZ).
    """
    J_h = np.asarray(J_h, np.float64)
    J_v = np.asarray(J_v, np.float64)
    L = J_h.shape[0]
    s = _row_spins(L)
    psis = [None] * L
    ls = np.zeros(L)

    def horiz(r):
        return np.exp(beta * (J_h[r][None, :] * s[:, :-1] * s[:, 1:]).sum(axis=1))

    psi = horiz(L - 1)
    n = np.linalg.norm(psi)
    psis[L - 1], ls[L - 1] = psi / n, math.log(n)
    for r in range(L - 2, -1, -1):
        mats = [np.exp(beta * J_v[r, c] * np.outer([-1.0, 1.0], [-1.0, 1.0])) for c in range(L)]
        psi = horiz(r) * _apply_site_matrices(psis[r + 1], mats)
        n0 = np.linalg.norm(psi)
        psi = psi / n0
        if chi is not None:
            # every second row mirrored, as the alternating compression does
            psi = _truncate_dense(psi, L, chi, alternate and (L - 2 - r) % 2 == 1)
        n1 = np.linalg.norm(psi)
        psis[r], ls[r] = psi / n1, math.log(n0) + math.log(n1)
    logZ = float(ls.sum() + math.log(psis[0].sum()))
    return psis, ls, logZ


def transfer_mean_energy(J_h, J_v, beta):
    """Exact <E> = -d ln Z / d beta, carrying (psi, d psi/d beta) row by row."""
    J_h = np.asarray(J_h, np.float64)
    J_v = np.asarray(J_v, np.float64)
    L = J_h.shape[0]
    s = _row_spins(L)
    ss = np.outer([-1.0, 1.0], [-1.0, 1.0])

    def horiz(r):
        e = (J_h[r][None, :] * s[:, :-1] * s[:, 1:]).sum(axis=1)   # = -E_h
        w = np.exp(beta * e)
        return w, e * w

    psi, dpsi = horiz(L - 1)
    for r in range(L - 2, -1, -1):
        t = psi.reshape((2,) * L)
        dt = dpsi.reshape((2,) * L)
        for c in range(L):
            B = np.exp(beta * J_v[r, c] * ss)
            dB = J_v[r, c] * ss * B
            nt = np.moveaxis(np.tensordot(B, t, axes=(1, c)), 0, c)
            ndt = (np.moveaxis(np.tensordot(dB, t, axes=(1, c)), 0, c)
                   + np.moveaxis(np.tensordot(B, dt, axes=(1, c)), 0, c))
            t, dt = nt, ndt
        w, dw = horiz(r)
        psi, dpsi = w * t.reshape(-1), dw * t.reshape(-1) + w * dt.reshape(-1)
        n = np.abs(psi).max()
        psi, dpsi = psi / n, dpsi / n
    return -float(dpsi.sum() / psi.sum())


def dense_row_logits(psi, L, beta, J_up, u_bits, row_bits):
    """Conditional logits of one row computed from its dense vector.

    psi: (2**L,) row vector; J_up (L,), u_bits (L,) the row above;
    row_bits (L,) the row's own spins (bits) defining each prefix.
    logit_c = ln|f_+| - ln|f_-| + 2 beta J_up(c) u_c with
    f_s = sum over the columns right of c of prod_{c'>c} B_up(c')[u, s_c'] psi.
    """
    J_up = np.asarray(J_up, np.float64)
    out = np.zeros(L)
    prefix = 0
    for c in range(L):
        t = psi.reshape(2 ** c, 2, 2 ** (L - c - 1))[prefix]           # (2, rest)
        w = np.ones(1)
        for cc in range(c + 1, L):
            B = np.exp(beta * J_up[cc] * np.outer([-1.0, 1.0], [-1.0, 1.0]))
            w = np.kron(w, B[u_bits[cc]])
        f = np.abs(t @ w)
        field = 2.0 * beta * J_up[c] * (2.0 * u_bits[c] - 1.0)
        with np.errstate(divide="ignore"):
            out[c] = math.log(f[1]) - math.log(f[0]) + field if f.min() > 0 else (
                math.inf if f[0] == 0 and f[1] > 0 else (-math.inf if f[1] == 0 and f[0] > 0 else 0.0))
        prefix = prefix * 2 + int(row_bits[c])
    return out


def iter_row_bits(L):
    return itertools.product((0, 1), repeat=L)
