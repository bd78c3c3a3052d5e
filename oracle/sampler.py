"""Row-by-row autoregressive sampler (oracle side, float64).

Test infrastructure only: nothing in the product path imports this module.

Follows section 3.3 (the row sampler and its four steps) with the chain rule
of Eq. (3) in raster order and the sigmoid form of Eq. (5):

for each row r (top to bottom) with the cached MPS A of row r and the spins u
of row r-1 (row 0 has no upper neighbour: its up-couplings are zero), the
conditional partition function of Eq. (4) at column c is the cached row
contracted with the chosen spins on its left, the candidate spin, and on its
right every spin summed with the weight of its bond to the row above.  The
right parts are accumulated once per row from the right end (one matrix per
sample: the site tensor summed over its spin with those weights); then the
columns are visited left to right, each one giving the two weights, the
logit of Eq. (5), the draw (or the given spin when teacher forcing), its
log-probability, and the left vector extended by the chosen spin.

Readings: environments are normalised by their 2-norm (any positive factor
cancels in rho_+/rho_-); log q is accumulated in float64; the uniform comes
from Philox4x32-10 with counter (r*L + c, sample, instance, 0).  If both rho
vanish the conditional is taken as 1/2.

Pins (tests/test_oracle_sampler.py): in the exact regime log q(s) equals
-beta E(s) - ln Z for every s (brute force); at any chi sum_s q(s) = 1; at
truncated chi the conditionals equal those computed from the dense
truncated states; Z2 symmetry.
"""
from __future__ import annotations

import numpy as np

from . import philox


def _log_sigmoid(x):
    """ln(1/(1+e^-x)) computed without overflow; x may be +-inf."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        out = -np.logaddexp(0.0, -x)
    return out


def _up_weights(beta, J_up, u_bits):
    """Boltzmann weight of each candidate spin through its bond to the row
    above (Eq. 7): w[n, c, s] = exp(beta J_up(c) sigma(u[n, c]) sigma(s)),
    with sigma(bit) = 2 bit - 1.  Shape (n, L, 2)."""
    su = 2.0 * np.asarray(u_bits, dtype=np.float64) - 1.0           # (n, L)
    ss = np.array([-1.0, 1.0])
    return np.exp(beta * J_up[None, :, None] * su[:, :, None] * ss[None, None, :])


def _unit_rows(v):
    """Each row of v divided by its 2-norm (a positive factor per sample)."""
    return v / np.sqrt((v * v).sum(axis=1, keepdims=True))


def sample_row(A, beta, J_up, u_bits, n, uniforms=None, forced_bits=None):
    """Sample (or score) one row for n configurations.

    A: list of L site tensors (Dl, 2, Dr) of this row's cache.
    J_up: (L,) couplings to the row above (zeros for row 0).
    u_bits: (n, L) bits of the row above (ignored where J_up is zero).
    uniforms: (n, L) uniforms for drawing; forced_bits: (n, L) to score.
    Returns (bits (n, L) int, logq (n,) float64, logits (n, L) float64).

    The conditional partition function of Eq. (4) for spin s at column c of
    this row, the spins left of c and the whole row above being fixed, is
    the cached row contracted with
      * the chosen spins at columns < c (the left vector l),
      * spin s at column c,
      * at every column c' > c the sum over its spin s' weighted by the
        bond to the row above, w(c', s') -- the right vector R_c,
    times w(c, s).  In the ratio of Eq. (5) the factor w(c, +)/w(c, -) is
    exp(2 beta J_up(c) sigma(u_c)), kept apart as a field term.
    """
    L = len(A)
    J_up = np.asarray(J_up, dtype=np.float64)
    w = _up_weights(beta, J_up, u_bits)
    # right vectors, built from the right end: R_{L-1} = [1] (the open end),
    # R_c = (sum_s w(c+1, s) A_{c+1}[:, s, :]) R_{c+1}, one matrix per sample
    R = [None] * L
    R[L - 1] = np.ones((n, 1))
    for c in range(L - 2, -1, -1):
        T = (w[:, c + 1, 0, None, None] * A[c + 1][None, :, 0, :]
             + w[:, c + 1, 1, None, None] * A[c + 1][None, :, 1, :])   # (n, Dl, Dr)
        R[c] = _unit_rows(np.matmul(T, R[c + 1][:, :, None])[:, :, 0])
    # left to right: probability, draw, log-probability, left-vector update
    left = np.ones((n, 1))
    bits = np.zeros((n, L), dtype=np.int64)
    logits = np.zeros((n, L))
    logq = np.zeros(n)
    for c in range(L):
        y = [left @ A[c][:, s, :] for s in (0, 1)]                      # l A_c[:, s, :]
        rho = [np.abs((y[s] * R[c]).sum(axis=1)) for s in (0, 1)]
        field = 2.0 * beta * J_up[c] * (2.0 * np.asarray(u_bits[:, c], np.float64) - 1.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.log(rho[1]) - np.log(rho[0]) + field
        lg = np.where(np.isnan(lg), 0.0, lg)                           # both zero: p = 1/2
        logits[:, c] = lg
        if forced_bits is not None:
            b = np.asarray(forced_bits[:, c], dtype=np.int64)
        else:
            with np.errstate(over="ignore"):
                p = 1.0 / (1.0 + np.exp(-lg))
            b = (uniforms[:, c] < p).astype(np.int64)
        bits[:, c] = b
        logq += np.where(b == 1, _log_sigmoid(lg), _log_sigmoid(-lg))
        left = _unit_rows(np.where(b[:, None] == 1, y[1], y[0]))
    return bits, logq, logits


def sample(cache, beta, J_v, n, seed=0, instance=0, sample_offset=0, forced_bits=None):
    """Sample n configurations of one instance from its cache.

    Returns (bits (n, L, L), logq (n,), logits (n, L, L)).  With forced_bits
    (n, L, L) the given configurations are scored instead (teacher forcing).
    """
    L = len(cache)
    J_v = np.asarray(J_v, dtype=np.float64)
    bits = np.zeros((n, L, L), dtype=np.int64)
    logits = np.zeros((n, L, L))
    logq = np.zeros(n)
    sample_idx = sample_offset + np.arange(n, dtype=np.uint64)
    for r in range(L):
        J_up = J_v[r - 1] if r > 0 else np.zeros(L)
        u = bits[:, r - 1] if r > 0 else np.zeros((n, L), dtype=np.int64)
        unif = None
        if forced_bits is None:
            site = (r * L + np.arange(L, dtype=np.uint64))[None, :]
            unif = philox.uniform(seed, site, sample_idx[:, None], instance,
                                  philox.STREAM_SITE)
        fb = None if forced_bits is None else np.asarray(forced_bits)[:, r]
        b, lq, lg = sample_row(cache[r], beta, J_up, u, n, unif, fb)
        bits[:, r], logits[:, r] = b, lg
        logq += lq
    return bits, logq, logits
