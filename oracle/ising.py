"""Ising spin-glass definitions (oracle side, float64).

Test infrastructure only: nothing in the product path imports this module.

* Energy, Eq. (1) of section 2.1: E(s) = -sum_<ij> J_ij s_i s_j over the
  nearest-neighbour bonds of the open L x L lattice, each bond counted once.
* Boltzmann matrix, Eq. (7) of section 2.2: B[a, b] = exp(beta * J * s_a * s_b)
  with index 0 <-> spin -1 and index 1 <-> spin +1 (the sampler of section 3.3
  maps a stored bit x to the spin 2x - 1).
* Spin packing into the 64-bit words the GPU path reads and writes.
"""
from __future__ import annotations

import numpy as np


def boltzmann_matrix(beta: float, J: float) -> np.ndarray:
    """Eq. (7): 2x2 matrix exp(beta*J*s_a*s_b), rows/cols ordered (-1, +1)."""
    s = np.array([-1.0, 1.0])
    return np.exp(float(beta) * float(J) * np.outer(s, s))


def energy(spins: np.ndarray, J_h: np.ndarray, J_v: np.ndarray) -> np.ndarray:
    """Eq. (1) for spins of shape (..., L, L) with values in {-1, +1}.

    Returns float64 of shape (...).  For couplings on the 2**-20 grid the
    float64 sum is exact whatever the summation order.
    """
    s = np.asarray(spins, dtype=np.float64)
    jh = np.asarray(J_h, dtype=np.float64)
    jv = np.asarray(J_v, dtype=np.float64)
    eh = (jh * s[..., :, :-1] * s[..., :, 1:]).sum(axis=(-1, -2))
    ev = (jv * s[..., :-1, :] * s[..., 1:, :]).sum(axis=(-1, -2))
    return -(eh + ev)


def bits_to_spins(bits: np.ndarray) -> np.ndarray:
    """{0, 1} -> {-1, +1}."""
    return 2 * np.asarray(bits, dtype=np.int64) - 1


def pack_spins(spins: np.ndarray) -> np.ndarray:
    """(..., L, L) spins in {-1,+1} -> (..., L, ceil(L/64)) uint64 words,
    bit (c mod 64) of word c//64 set iff spin (r, c) is +1."""
    s = np.asarray(spins)
    L = s.shape[-1]
    W = (L + 63) // 64
    out = np.zeros(s.shape[:-1] + (W,), dtype=np.uint64)
    up = (s > 0)
    for c in range(L):
        out[..., c // 64] |= up[..., c].astype(np.uint64) << np.uint64(c % 64)
    return out


def unpack_spins(words: np.ndarray, L: int) -> np.ndarray:
    """Inverse of pack_spins."""
    w = np.asarray(words, dtype=np.uint64)
    out = np.empty(w.shape[:-1] + (L,), dtype=np.int8)
    for c in range(L):
        bit = (w[..., c // 64] >> np.uint64(c % 64)) & np.uint64(1)
        out[..., c] = np.where(bit == 1, 1, -1)
    return out
