"""Boundary-MPS cache build (oracle side, float64, dense).

Test infrastructure only: nothing in the product path imports this module.

Follows section 3.2 (cache initialization) and section 2.2 (Eqs. (6)-(8),
Fig. 2) step by step, with plain dense tensors:

1. bottom row L-1: the product of that row's horizontal Boltzmann weights
   as a bond-dimension-2 MPS, every bond carrying the spin its Boltzmann
   matrix passes on (site shapes (1,2,2), (2,2,2), ..., (2,2,1));
2. for each row r = L-2 ... 0: the row's transfer operator as an MPO whose
   entries are written out from Eqs. (7)-(8) (index order left, own spin,
   right, lower spin; shapes (1,2,2,2), (2,2,2,2), ..., (2,2,1,2)); apply it
   to the MPS ("multiply", which doubles the bond); truncate back to chi
   ("compress").

``compress`` is not listed in the paper; the reading used here (and by the
GPU path) is: a left-to-right QR sweep that makes every site left-canonical
(exact, no truncation), then a right-to-left SVD sweep that at each bond keeps
the min(chi, rank-bound) largest singular values, with no relative cutoff.
Every norm taken out is accumulated in a float64 log-scale, so that

    ln Z_TN = sum_r logscale[r] + ln( prod_c sum_s A^(0)_c[:, s, :] ).

The cache row r represents, up to the scale exp(sum_{r' >= r} logscale[r']),
the function of row r's spins  psi_r(s_r) = sum over rows > r of
exp(-beta * E(rows >= r)), i.e. it includes row r's horizontal bonds and every
vertical bond below row r (exactly when chi >= 2**floor(L/2)).

Pins (tests/test_oracle_bmps.py): brute-force ln Z on 3x3/4x4, the dense
transfer vector (exact and with the same sequential truncation) on L <= 10,
closed forms (J_v = 0, J_h = 0, beta = 0) at large L, Z2 and gauge invariance.
The cut diagnostic of compress is pinned on states with a prescribed
Schmidt spectrum (tests/test_oracle_exact.py).
"""
from __future__ import annotations

import math

import numpy as np

from .ising import boltzmann_matrix


def _normalise(t: np.ndarray):
    nu = float(np.linalg.norm(t))
    return t / nu, math.log(nu)


def _bond_dims(L: int, c: int):
    """(left, right) bond dimensions of column c in a bond-2 row network:
    the open ends carry a trivial index of dimension 1."""
    return (1 if c == 0 else 2), (1 if c == L - 1 else 2)


def bottom_row_mps(beta: float, J_h: np.ndarray):
    """Row L-1 of the cache, bond dimension 2 (section 3.2).

    The bottom row's function of its spins is the product of its horizontal
    Boltzmann weights (Eq. 7), psi(s) = prod_c B(J_h[L-1, c])[s_c, s_{c+1}].
    Written as an MPS, the bond between columns c and c+1 carries the spin
    reached through that bond's Boltzmann matrix, and the copy tensor of
    Eq. (8) at column c+1 forces it to equal s_{c+1}:

        A_c[a, s, b] = [c == 0 or a == s] * (B_c[s, b] if c < L-1 else 1).
    """
    L = J_h.shape[0]
    mps = []
    for c in range(L):
        Dl, Dr = _bond_dims(L, c)
        Bh = boltzmann_matrix(beta, J_h[L - 1, c]) if c < L - 1 else None
        A = np.zeros((Dl, 2, Dr))
        for a in range(Dl):
            for s in range(2):
                if c > 0 and a != s:
                    continue                      # copy tensor: left bond = own spin
                for b in range(Dr):
                    A[a, s, b] = Bh[s, b] if Bh is not None else 1.0
        mps.append(A)
    # Scale each site to unit norm; the state changes only by a positive
    # factor, which is kept in the log-scale.
    logscale = 0.0
    for c in range(L):
        mps[c], ln = _normalise(mps[c])
        logscale += ln
    return mps, logscale


def row_mpo(beta: float, J_h: np.ndarray, J_v: np.ndarray, row: int):
    """Transfer MPO of one row (section 3.2, Eqs. 7-8).

    The row's spins s_c interact with their right neighbours through
    B(J_h[row, c]) and with the spins n_c of the row below through
    B(J_v[row, c]).  As an operator from the lower row's spins n to the
    row's own spins s, with a bond index carrying s_c's horizontal weight to
    column c+1 (where the copy tensor makes it equal s_{c+1}):

        W_c[l, s, r, n] = [c == 0 or l == s]
                          * (B(J_h[row, c])[s, r] if c < L-1 else 1)
                          * B(J_v[row, c])[s, n].

    Index order (left, own spin, right, lower spin); the open ends have
    dimension 1.
    """
    L = J_h.shape[0]
    mpo = []
    for c in range(L):
        Dl, Dr = _bond_dims(L, c)
        Bh = boltzmann_matrix(beta, J_h[row, c]) if c < L - 1 else None
        Bv = boltzmann_matrix(beta, J_v[row, c])
        W = np.zeros((Dl, 2, Dr, 2))
        for l in range(Dl):
            for s in range(2):
                if c > 0 and l != s:
                    continue
                for r in range(Dr):
                    h = Bh[s, r] if Bh is not None else 1.0
                    for n in range(2):
                        W[l, s, r, n] = h * Bv[s, n]
        mpo.append(W)
    return mpo


def multiply(mpo, mps):
    """MPO x MPS: new[(a,l), s, (b,r)] = sum_n W[l, s, r, n] A[a, n, b]."""
    out = []
    for W, A in zip(mpo, mps):
        Dl, _, Dr = A.shape
        wl, _, wr, _ = W.shape
        t = np.einsum("lsrn,anb->alsbr", W, A)
        out.append(t.reshape(Dl * wl, 2, Dr * wr))
    return out


def mirror(mps):
    """The same state with the column order reversed: site c becomes site
    L-1-c and its left and right bonds trade places."""
    return [np.transpose(t, (2, 1, 0)).copy() for t in reversed(mps)]


def row_is_mirrored(L: int, row: int, alternate: bool) -> bool:
    """With alternating sweeps, the rows compressed second, fourth, ... from
    the bottom (row L-3, L-5, ...) are compressed right to left."""
    return alternate and (L - 2 - row) % 2 == 1


def compress(mps, chi: int, diag=None):
    """QR sweep left->right, then truncating SVD sweep right->left.

    Returns (log of the norms taken out, new list of sites).  Bond c|c+1 ends
    with dimension min(chi, rank bound); the singular values kept are the
    largest ones, with no cutoff.  If `diag` is a dict, diag["cond"] is raised
    to the largest sigma_k / (sigma_k - sigma_{k+1}) over the cuts that
    discard something (sigma_k above 1e-13 sigma_1): the factor by which
    rounding is amplified in the truncated state when the cut falls inside a
    near-degenerate pair (infinite for an exact tie).
    """
    mps = [t.copy() for t in mps]
    L = len(mps)
    logn = 0.0
    for c in range(L - 1):
        Dl, d, Dr = mps[c].shape
        Q, R = np.linalg.qr(mps[c].reshape(Dl * d, Dr), mode="reduced")
        R, ln = _normalise(R)
        logn += ln
        mps[c] = Q.reshape(Dl, d, Q.shape[1])
        mps[c + 1] = np.tensordot(R, mps[c + 1], axes=(1, 0))
    mps[L - 1], ln = _normalise(mps[L - 1])
    logn += ln
    for c in range(L - 1, 0, -1):
        Dl, d, Dr = mps[c].shape
        U, S, Vt = np.linalg.svd(mps[c].reshape(Dl, d * Dr), full_matrices=False)
        k = min(chi, S.shape[0])
        if diag is not None and k < S.shape[0] and S[k - 1] > 1e-13 * S[0]:
            gap = S[k - 1] - S[k]
            diag["cond"] = max(diag.get("cond", 0.0), S[k - 1] / gap if gap > 0 else math.inf)
        U, S, Vt = U[:, :k], S[:k], Vt[:k]
        nrm = float(np.linalg.norm(S))
        logn += math.log(nrm)
        mps[c] = Vt.reshape(k, d, Dr)
        mps[c - 1] = np.tensordot(mps[c - 1], U * (S / nrm), axes=(2, 0))
    mps[0], ln = _normalise(mps[0])
    logn += ln
    return logn, mps


def build_cache(beta: float, J_h: np.ndarray, J_v: np.ndarray, chi: int, diag=None, alternate: bool = False):
    """The full cache for one instance.

    Returns (cache, logscale, logZ) where cache[r] is the list of row r's
    site tensors (shapes (Dl, 2, Dr), normalised), logscale[r] the log of the
    norms taken out when row r was formed, and logZ the TN estimate of ln Z.
    `diag` (optional dict) collects the truncation conditioning, see compress.
    With `alternate`, every second row (row_is_mirrored) is compressed in
    the mirrored orientation -- QR sweep right to left, truncating SVD sweep
    left to right -- an equally canonical compression (compress is not
    listed in the paper) whose sites come out in the order the next row's
    QR sweep consumes them.
    """
    J_h = np.asarray(J_h, dtype=np.float64)
    J_v = np.asarray(J_v, dtype=np.float64)
    L = J_h.shape[0]
    cache = [None] * L
    logscale = np.zeros(L)
    mps, logscale[L - 1] = bottom_row_mps(beta, J_h)
    cache[L - 1] = mps
    for row in range(L - 2, -1, -1):
        mps = multiply(row_mpo(beta, J_h, J_v, row), mps)
        if row_is_mirrored(L, row, alternate):
            logscale[row], mps = compress(mirror(mps), chi, diag)
            mps = mirror(mps)
        else:
            logscale[row], mps = compress(mps, chi, diag)
        cache[row] = mps
    return cache, logscale, float(logscale.sum() + log_total(cache[0]))


def log_total(mps) -> float:
    """ln of the MPS contracted with every physical index summed."""
    v = np.ones(1)
    lsum = 0.0
    for A in mps:
        v = v @ A.sum(axis=1)
        n = float(np.abs(v).max())
        v = v / n
        lsum += math.log(n)
    return lsum + math.log(float(v[0]))


def mps_to_dense(mps) -> np.ndarray:
    """Dense 2**L vector of an MPS, spin index 0 of site 0 most significant."""
    v = mps[0].reshape(2, -1)
    for A in mps[1:]:
        Dl, _, Dr = A.shape
        v = (v @ A.reshape(Dl, 2 * Dr)).reshape(-1, Dr)
    return v.reshape(-1)
