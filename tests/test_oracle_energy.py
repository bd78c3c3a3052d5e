"""Pins for the oracle energy (Eq. 1) and spin packing."""
import math

import numpy as np

import workloads
from oracle import exact, ising


def test_ferromagnet_ground_state():
    L = 7
    jh, jv = np.ones((L, L - 1)), np.ones((L - 1, L))
    up = np.ones((L, L), dtype=np.int8)
    assert ising.energy(up, jh, jv) == -2 * L * (L - 1)
    checker = np.where((np.add.outer(np.arange(L), np.arange(L)) % 2) == 0, 1, -1)
    assert ising.energy(checker, jh, jv) == 2 * L * (L - 1)


def test_spin_flip_symmetry_and_integers():
    jh, jv = workloads.instance(9, "pmj", 5, 0)
    s = workloads.random_spins(20, 9, 1)
    e = ising.energy(s, jh, jv)
    assert np.array_equal(e, ising.energy(-s, jh, jv))
    assert np.array_equal(e, np.round(e))


def test_single_flip_equals_local_field():
    """E(s with s_i flipped) - E(s) = 2 s_i h_i, h_i = sum of J s over the
    neighbours of i: a local statement independent of the global sum."""
    L = 6
    jh, jv = workloads.instance(L, "gauss", 5, 1)
    s = workloads.random_spins(1, L, 2)[0].astype(np.int64)
    e0 = ising.energy(s, jh, jv)
    for r in range(L):
        for c in range(L):
            h = 0.0
            if c > 0:
                h += jh[r, c - 1] * s[r, c - 1]
            if c < L - 1:
                h += jh[r, c] * s[r, c + 1]
            if r > 0:
                h += jv[r - 1, c] * s[r - 1, c]
            if r < L - 1:
                h += jv[r, c] * s[r + 1, c]
            t = s.copy()
            t[r, c] = -t[r, c]
            assert ising.energy(t, jh, jv) - e0 == 2 * s[r, c] * h


def test_matches_bond_by_bond_enumeration():
    for L, fam in ((3, "pmj"), (4, "gauss")):
        jh, jv = workloads.instance(L, fam, 3, 0)
        e1 = ising.energy(exact.all_configs(L), jh, jv)
        e2 = exact.brute_energies(jh.astype(np.float64), jv.astype(np.float64))
        assert np.array_equal(e1, e2)


def test_grid_couplings_sum_exactly_in_any_order():
    L = 64
    jh, jv = workloads.instance(L, "gauss", 7, 0)
    assert np.all(np.abs(jh) < 8) and np.all(np.abs(jv) < 8)
    assert np.array_equal(jh.astype(np.float64) * 2 ** 20, np.round(jh.astype(np.float64) * 2 ** 20))
    s = workloads.random_spins(1, L, 3)[0].astype(np.float64)
    terms = np.concatenate([(jh * s[:, :-1] * s[:, 1:]).ravel(), (jv * s[:-1] * s[1:]).ravel()])
    ref = -math.fsum(terms)
    rng = np.random.default_rng(0)
    for _ in range(5):
        acc = 0.0
        for t in rng.permutation(terms):
            acc += t
        assert -acc == ref
    assert ising.energy(s, jh, jv) == ref


def test_pack_roundtrip():
    for L in (5, 64, 65, 130):
        s = workloads.random_spins(3, L, L)
        w = ising.pack_spins(s)
        assert w.shape == (3, L, (L + 63) // 64) and w.dtype == np.uint64
        assert np.array_equal(ising.unpack_spins(w, L), s)
    s = np.ones((1, 1, 3), dtype=np.int8)
    assert int(ising.pack_spins(s)[0, 0, 0]) == 0b111
