"""Seeded synthetic spin-glass instances (couplings only).

This module is the one piece shared by the CPU oracle and the GPU path: it
draws coupling arrays and holds none of the sampling method's arithmetic.

Couplings follow the open-boundary square lattice of the paper (section 3.1):
every nearest-neighbour bond appears once,

* ``J_h[r, c]`` couples site (r, c) with (r, c+1), shape (L, L-1);
* ``J_v[r, c]`` couples site (r, c) with (r+1, c), shape (L-1, L).

Two coupling families are provided:

* ``"pmj"``   -- the Edwards-Anderson +-J model, J = -1 with probability p
  (p = 0.5 is the EA spin glass used for the paper's results, section 4);
* ``"gauss"`` -- Gaussian N(0, 1) couplings rounded to multiples of 2**-20
  and clipped to |J| < 8.  On that grid every coupling is exact in float32
  and every partial energy sum is an integer multiple of 2**-20 far below
  2**53, so energies summed in float64 are exact in any order.

Instances are drawn with numpy's PCG64 seeded by (family tag, config id,
instance index), so each instance is reproducible on its own.
"""
from __future__ import annotations

import numpy as np

GRID = 2.0 ** -20
JMAX = 8.0 - GRID
_FAMILY_TAG = {"pmj": 1, "gauss": 2}


def _rng(family: str, config_id: int, index: int) -> np.random.Generator:
    return np.random.default_rng(
        np.random.SeedSequence([0x7E4C, _FAMILY_TAG[family], int(config_id), int(index)]))


def instance(L: int, family: str = "pmj", config_id: int = 0, index: int = 0,
             p: float = 0.5):
    """One instance: (J_h float32 (L, L-1), J_v float32 (L-1, L))."""
    if L < 2:
        raise ValueError("L must be >= 2")
    rng = _rng(family, config_id, index)
    nh, nv = L * (L - 1), (L - 1) * L
    if family == "pmj":
        neg = rng.random(nh + nv) < p
        j = np.where(neg, -1.0, 1.0)
    elif family == "gauss":
        g = rng.standard_normal(nh + nv)
        j = np.clip(np.round(g / GRID) * GRID, -JMAX, JMAX)
    else:
        raise ValueError(f"unknown coupling family {family!r}")
    j = j.astype(np.float32)
    return j[:nh].reshape(L, L - 1).copy(), j[nh:].reshape(L - 1, L).copy()


def batch(L: int, n: int, family: str = "pmj", config_id: int = 0, first: int = 0,
          p: float = 0.5):
    """n instances of one size: (J_h (n, L, L-1), J_v (n, L-1, L)) float32."""
    jh = np.empty((n, L, L - 1), np.float32)
    jv = np.empty((n, L - 1, L), np.float32)
    for i in range(n):
        jh[i], jv[i] = instance(L, family, config_id, first + i, p)
    return jh, jv


def betas_uniform(n: int, lo: float, hi: float, config_id: int = 0) -> np.ndarray:
    """Per-instance inverse temperatures drawn uniformly in [lo, hi]."""
    rng = np.random.default_rng(np.random.SeedSequence([0x7E4C, 9, int(config_id)]))
    return lo + (hi - lo) * rng.random(n)


def random_spins(n: int, L: int, seed: int = 0) -> np.ndarray:
    """Uniformly random spin configurations in {-1, +1}, shape (n, L, L) int8."""
    rng = np.random.default_rng(np.random.SeedSequence([0x5B1D, int(seed)]))
    return np.where(rng.random((n, L, L)) < 0.5, -1, 1).astype(np.int8)


def uneven_mix(n: int = 512, config_id: int = 4):
    """The uneven batch: sizes cycle through {32, 64, 128, 256}; coupling family
    alternates in blocks of four (+-J, then Gaussian); bond dimension cycles
    through {16, 32, 64} in blocks of eight; beta uniform in [0.5, 2.0].

    Returns a list of dicts with keys L, family, chi, beta, J_h, J_v.
    """
    betas = betas_uniform(n, 0.5, 2.0, config_id)
    out = []
    for i in range(n):
        L = (32, 64, 128, 256)[i % 4]
        family = "pmj" if (i // 4) % 2 == 0 else "gauss"
        chi = (16, 32, 64)[(i // 8) % 3]
        jh, jv = instance(L, family, config_id, i)
        out.append(dict(L=L, family=family, chi=chi, beta=float(betas[i]), J_h=jh, J_v=jv))
    return out
