"""Pins for the oracle boundary-MPS build (section 3.2, Eqs. 6-8)."""
import math

import numpy as np
import pytest

import workloads
from oracle import bmps, exact


@pytest.mark.parametrize("L,fam", [(3, "pmj"), (3, "gauss"), (4, "pmj"), (4, "gauss")])
@pytest.mark.parametrize("beta", [0.3, 1.0, 2.0])
def test_exact_regime_equals_brute_force(L, fam, beta):
    jh, jv = workloads.instance(L, fam, 11, 0)
    _, _, lz = bmps.build_cache(beta, jh, jv, chi=2 ** (L // 2))
    assert abs(lz - exact.brute_logZ(jh, jv, beta)) < 1e-12 * max(1.0, abs(lz))


@pytest.mark.parametrize("L", [6, 8])
def test_exact_regime_equals_transfer_vector(L):
    jh, jv = workloads.instance(L, "gauss", 12, 0)
    _, _, lz = bmps.build_cache(1.0, jh, jv, chi=2 ** (L // 2))
    _, _, tz = exact.transfer_vectors(jh, jv, 1.0)
    assert abs(lz - tz) < 1e-11 * abs(tz)


def test_below_exact_chi_is_not_exact():
    jh, jv = workloads.instance(6, "gauss", 12, 1)
    _, _, tz = exact.transfer_vectors(jh, jv, 1.0)
    _, _, lz4 = bmps.build_cache(1.0, jh, jv, chi=4)
    _, _, lz8 = bmps.build_cache(1.0, jh, jv, chi=8)
    assert abs(lz8 - tz) < 1e-11 * abs(tz)
    assert abs(lz4 - tz) > 1e-8


@pytest.mark.parametrize("alternate", [False, True])
@pytest.mark.parametrize("L,chi", [(6, 2), (6, 3), (8, 3), (8, 5)])
def test_truncated_equals_dense_sequential_truncation(L, chi, alternate):
    """At truncated chi, every cached row equals the dense row vector with
    the same Schmidt truncation (right-to-left; with alternating sweeps every
    second row left-to-right), and ln Z agrees."""
    jh, jv = workloads.instance(L, "pmj", 13, L + chi)
    cache, ls, lz = bmps.build_cache(1.0, jh, jv, chi, alternate=alternate)
    psis, tls, tz = exact.transfer_vectors(jh, jv, 1.0, chi=chi, alternate=alternate)
    assert abs(lz - tz) < 1e-10 * abs(tz)
    for r in range(L):
        v = bmps.mps_to_dense(cache[r])
        nv = np.linalg.norm(v)
        v = v * np.sign(v @ psis[r]) / nv
        assert np.abs(v - psis[r]).max() < 1e-10
        # psi_r = exp(cumulative log-scale) * state: compare the total norm
        lhs = ls[r:].sum() + np.log(nv)
        rhs = tls[r:].sum()
        assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(rhs))


def test_bond_dimensions_follow_rank_bound():
    L, chi = 9, 4
    jh, jv = workloads.instance(L, "gauss", 14, 0)
    cache, _, _ = bmps.build_cache(1.0, jh, jv, chi)
    for r in range(L - 1):
        dims = [A.shape[2] for A in cache[r][:-1]]
        assert dims == [min(chi, 2 ** min(b + 1, L - 1 - b)) for b in range(L - 1)]


def test_closed_form_no_vertical_bonds():
    """J_v = 0: rows are independent open chains, Z = prod_rows 2 prod_c 2cosh(beta J)."""
    L, beta = 40, 1.3
    jh, _ = workloads.instance(L, "gauss", 15, 0)
    jv = np.zeros((L - 1, L), np.float32)
    _, _, lz = bmps.build_cache(beta, jh, jv, chi=2)
    want = L * math.log(2) + np.log(2 * np.cosh(beta * jh.astype(np.float64))).sum()
    assert abs(lz - want) < 1e-11 * abs(want)


def test_closed_form_no_horizontal_bonds():
    L, beta = 24, 0.9
    _, jv = workloads.instance(L, "pmj", 15, 1)
    jh = np.zeros((L, L - 1), np.float32)
    _, _, lz = bmps.build_cache(beta, jh, jv, chi=1)
    want = L * math.log(2) + np.log(2 * np.cosh(beta * jv.astype(np.float64))).sum()
    assert abs(lz - want) < 1e-11 * abs(want)


def test_infinite_temperature():
    L = 20
    jh, jv = workloads.instance(L, "gauss", 15, 2)
    _, _, lz = bmps.build_cache(0.0, jh, jv, chi=3)
    assert abs(lz - L * L * math.log(2)) < 1e-10 * L * L


def test_mattis_gauge_invariance_at_truncated_chi():
    """J'_ij = xi_i xi_j J_ij is a relabelling of spins: ln Z is unchanged at
    any chi because the truncation only sees singular values."""
    L, chi = 10, 3
    jh, jv = workloads.instance(L, "gauss", 16, 0)
    xi = workloads.random_spins(1, L, 9)[0].astype(np.float64)
    jh2 = (jh * xi[:, :-1] * xi[:, 1:]).astype(np.float32)
    jv2 = (jv * xi[:-1, :] * xi[1:, :]).astype(np.float32)
    _, _, a = bmps.build_cache(1.0, jh, jv, chi)
    _, _, b = bmps.build_cache(1.0, jh2, jv2, chi)
    assert abs(a - b) < 1e-11 * abs(a)


def test_truncated_total_can_be_non_positive():
    """At chi = 2 the truncated network is not a positive function: for this
    +-J 64x64 instance at beta 1.5 its total (every spin of row 0 summed) is
    not positive, so ln Z_TN is undefined (the GPU path reports the same,
    test_gpu_parity.py)."""
    import pytest
    import workloads
    jh, jv = workloads.instance(64, "pmj", 9, 13)
    with pytest.raises(ValueError):
        bmps.build_cache(1.5, jh, jv, 2)


def test_alternating_sweeps_change_only_the_truncation():
    """The mirrored compression is another canonical truncation: in the
    exact regime both orders give the same ln Z to rounding; truncated, they
    differ (at the truncation error) -- so oracle and kernel must agree on
    the order."""
    jh, jv = workloads.instance(8, "gauss", 14, 0)
    _, _, a = bmps.build_cache(1.0, jh, jv, 16)
    _, _, b = bmps.build_cache(1.0, jh, jv, 16, alternate=True)
    assert abs(a - b) < 1e-12 * abs(a)
    _, _, a = bmps.build_cache(1.0, jh, jv, 2)
    _, _, b = bmps.build_cache(1.0, jh, jv, 2, alternate=True)
    assert abs(a - b) > 1e-9 * abs(a)


def test_mirror_is_an_involution_and_keeps_the_state():
    jh, jv = workloads.instance(6, "pmj", 15, 0)
    mps, _ = bmps.bottom_row_mps(1.0, jh)
    v = bmps.mps_to_dense(mps).reshape((2,) * 6)
    w = bmps.mps_to_dense(bmps.mirror(mps)).reshape((2,) * 6)
    assert np.allclose(w, v.transpose(5, 4, 3, 2, 1, 0))
    back = bmps.mirror(bmps.mirror(mps))
    assert all(np.array_equal(x, y) for x, y in zip(back, mps))
