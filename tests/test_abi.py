"""The C ABI without a GPU: every declared symbol is exported, and argument
validation returns the documented status codes before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2509_19006_amd as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tnmc.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tnmc_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtnmc.so not built")
    return T.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "tnmc_build_env" in names and "tnmc_accept" in names and len(names) >= 13
    raw = ctypes.CDLL(T.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    assert set(T.EXPORTS) <= set(names)


def _problem(L=(8,), chi=(16,), beta=(1.0,)):
    return T.Problem(None, None, list(L), list(chi), list(beta))


@pytest.mark.parametrize("L,chi,beta,code", [
    ((1,), (4,), (1.0,), T.TNMC_EINVAL),
    ((2000,), (4,), (1.0,), T.TNMC_EINVAL),
    ((8,), (1,), (1.0,), T.TNMC_EINVAL),
    ((8,), (65,), (1.0,), T.TNMC_EINVAL),
    ((8,), (4,), (-1.0,), T.TNMC_EINVAL),
    ((8,), (4,), (float("nan"),), T.TNMC_EINVAL),
    ((8, 8), (4, 40), (1.0, 1.0), T.TNMC_ENOTSUP),    # float64 keeps chi <= 32
])
def test_workspace_size_validation(lib, L, chi, beta, code):
    with pytest.raises(T.TnmcError) as e:
        T.tnmc_workspace_size(_problem(L, chi, beta), T.FP64, 16)
    assert e.value.code == code
    assert len(lib.tnmc_last_error()) > 0


def test_workspace_grows_with_samples_and_tiles(lib):
    p = _problem((16, 33), (8, 8), (1.0, 0.5))
    a = T.tnmc_workspace_size(p, T.FP32, 1)
    b = T.tnmc_workspace_size(p, T.FP32, 256)
    c = T.tnmc_workspace_size(p, T.FP32, 257)
    assert a == b < c
    assert T.tnmc_workspace_size(p, T.FP64, 1) > a > T.tnmc_workspace_size(p, T.MIXED_BF16, 1)
    with pytest.raises(T.TnmcError):
        T.tnmc_workspace_size(p, 7, 1)
    with pytest.raises(T.TnmcError):
        T.tnmc_workspace_size(p, T.FP32, 0)


def test_entry_points_reject_bad_arguments_before_device_work(lib):
    P = ctypes.POINTER
    env = ctypes.c_void_p(0)
    p = _problem()
    # no couplings
    assert lib.tnmc_build_env(ctypes.byref(p._c), T.FP32, ctypes.c_void_p(256), 1 << 30, None,
                              ctypes.byref(env), None) == T.TNMC_EINVAL
    assert lib.tnmc_sample(None, 4, 0, 0, None, None, None, None, None, None) == T.TNMC_EINVAL
    assert lib.tnmc_energy(None, 4, None, None, None, None) == T.TNMC_EINVAL
    assert lib.tnmc_env_check(None, None) == T.TNMC_EINVAL
    assert lib.tnmc_accept(0, 4, None, None, None, None, 0, 0, None, None, None) == T.TNMC_EINVAL
    assert lib.tnmc_accept(2, 4, None, None, None, None, 0, 0, None, None, None) == T.TNMC_EINVAL
    assert lib.tnmc_philox_uniform(0, None, 0, 0, 0, 4, None, None) == T.TNMC_EINVAL
    assert lib.tnmc_mlp_train_step(None, None, None, 8, None, None, None, 1e-3, 1, None, None, None,
                                   None) == T.TNMC_EINVAL
    assert lib.tnmc_mlp_forward(None, 8, None, 0, None, None) == T.TNMC_EINVAL
    assert lib.tnmc_mlp_features(None, 8, None, None, None, None) == T.TNMC_EINVAL
    assert lib.tnmc_env_stats(None) is None
    assert lib.tnmc_mlp_scratch_floats(100) == 2 * T.MLP_NPARAM + 2
    assert lib.tnmc_mlp_scratch_floats(0) == 0


def test_chain_state_decoding():
    raw = np.zeros(2 * T.CHAIN_BYTES, dtype=np.uint8)
    f = raw.view(np.float64).reshape(2, 6)
    i = raw.view(np.int64).reshape(2, 6)
    f[1, 0], f[1, 1] = -3.5, 12.0
    i[1, 2], i[1, 3], i[1, 4], i[1, 5] = 41, 7, 40, 1
    st = T.chain_state(raw)
    assert st[1] == dict(cur_logq=-3.5, cur_E=12.0, cur_index=41, n_acc=7, n_trials=40, initialised=1)


def test_workspace_bytes_matches_status_form(lib):
    p = _problem((16, 33), (8, 8), (1.0, 0.5))
    assert T.tnmc_workspace_bytes(p, T.FP32, 300) == T.tnmc_workspace_size(p, T.FP32, 300) > 0
    # a bad problem gives 0 and an error text
    assert T.tnmc_workspace_bytes(_problem((1,), (4,), (1.0,)), T.FP32, 8) == 0
    assert b"L must be" in lib.tnmc_last_error()
    assert T.tnmc_workspace_bytes(p, T.FP32, 0) == 0


def test_coupling_kind_is_validated(lib):
    p = T.Problem(None, None, [8], [8], [1.0], coupling_kind=7)
    with pytest.raises(T.TnmcError) as e:
        T.tnmc_workspace_size(p, T.FP32, 8)
    assert e.value.code == T.TNMC_EINVAL


def test_problem_flags_are_validated(lib):
    for flags in (T.ALTERNATE_SWEEPS, T.FORCE_F64_FALLBACK, T.ALTERNATE_SWEEPS | T.FORCE_F64_FALLBACK,
                  T.ALTERNATE_SWEEPS | T.SHORT_WAITS):
        p = T.Problem(None, None, [8], [8], [1.0], flags=flags)
        assert T.tnmc_workspace_size(p, T.FP32, 8) > 0
    p = T.Problem(None, None, [8], [8], [1.0], flags=4)
    with pytest.raises(T.TnmcError) as e:
        T.tnmc_workspace_size(p, T.FP32, 8)
    assert e.value.code == T.TNMC_EINVAL


def test_float_builds_reserve_the_float64_redo_area(lib):
    """The workspace layout, written out for one instance: descriptor table,
    launch order, build statistics, then log-scales, cache, build scratch
    (Q slots and, in a float build, the float64 redo area: two blocks and
    their rotations of (chi+1)^2 doubles each, 256 doubles of rotations in
    flight, 2(chi+2) singular values), the parity-basis ping-pong, and one
    sampler tile of right environments (256 samples); every part aligned to
    256 bytes."""
    up = lambda x: (x + 255) // 256 * 256
    L, chi = 16, 8

    def expect(ts, ss, redo):
        fixed = up(96) + up(4) + up(8 * 16)
        fixed += up(8 * L) + up(L * L * 2 * chi * chi * ss) + up(L * 4 * chi * chi * ts + redo)
        fixed += up(2 * L * 2 * chi * chi * ts)
        return fixed + up(256 * L * 16 * ts)

    p = _problem((L,), (chi,), (1.0,))
    redo = 8 * (4 * (chi + 1) ** 2 + 256 + 2 * (chi + 2))
    assert T.tnmc_workspace_bytes(p, T.FP32, 8) == expect(4, 4, redo)
    assert T.tnmc_workspace_bytes(p, T.MIXED_FP16, 8) == expect(4, 2, redo)
    assert T.tnmc_workspace_bytes(p, T.FP64, 8) == expect(8, 8, 0)


def test_pipelined_build_doubles_the_q_slots(lib):
    """With alternating sweeps a float build of chi <= 32 pipelines its rows
    and keeps two rows of Q slots; float64 builds, and batches with chi > 32,
    keep one."""
    up = lambda x: (x + 255) // 256 * 256
    L, chi = 16, 8
    qrow = L * 4 * chi * chi * 4
    redo = 8 * (4 * (chi + 1) ** 2 + 256 + 2 * (chi + 2))
    plain = T.Problem(None, None, [L], [chi], [1.0])
    alt = T.Problem(None, None, [L], [chi], [1.0], flags=T.ALTERNATE_SWEEPS)
    d32 = T.tnmc_workspace_bytes(alt, T.FP32, 8) - T.tnmc_workspace_bytes(plain, T.FP32, 8)
    assert d32 == up(2 * qrow + redo) - up(qrow + redo)
    assert T.tnmc_workspace_bytes(alt, T.FP64, 8) == T.tnmc_workspace_bytes(plain, T.FP64, 8)
    wide = T.Problem(None, None, [L, L], [chi, 40], [1.0, 1.0], flags=T.ALTERNATE_SWEEPS)
    wide0 = T.Problem(None, None, [L, L], [chi, 40], [1.0, 1.0])
    assert T.tnmc_workspace_bytes(wide, T.FP32, 8) == T.tnmc_workspace_bytes(wide0, T.FP32, 8)


def _fake_problem(L, kind):
    """A problem whose device pointers are never dereferenced (the calls
    below fail validation before any device work)."""
    p = T.Problem(None, None, list(L), [8] * len(L), [1.0] * len(L), coupling_kind=kind)
    p._c.J_h = ctypes.c_void_p(256)
    p._c.J_v = ctypes.c_void_p(512)
    return p


def test_energy_validation(lib):
    fake = ctypes.c_void_p(1024)
    # the int32 output needs +-J couplings
    for kind in (T.COUPLING_GENERAL, T.COUPLING_GRID20):
        p = _fake_problem((8, 8), kind)
        assert lib.tnmc_energy(ctypes.byref(p._c), 4, fake, fake, fake, None) == T.TNMC_EINVAL
        assert b"COUPLING_PMJ" in lib.tnmc_last_error()
    p = _fake_problem((8, 1), T.COUPLING_PMJ)
    assert lib.tnmc_energy(ctypes.byref(p._c), 4, fake, fake, fake, None) == T.TNMC_EINVAL
    p = _fake_problem((8,), T.COUPLING_PMJ)
    assert lib.tnmc_energy(ctypes.byref(p._c), 0, fake, fake, fake, None) == T.TNMC_EINVAL
    assert lib.tnmc_energy(ctypes.byref(p._c), 4, None, fake, None, None) == T.TNMC_EINVAL


def test_philox_counter_overflow_is_rejected(lib):
    fake = ctypes.c_void_p(1024)
    # 2^32 - 4 + 8 proposals would wrap the 32-bit proposal counter
    rc = lib.tnmc_accept(2, 8, fake, fake, fake, fake, 0, (1 << 32) - 4, fake, None, None)
    assert rc == T.TNMC_EINVAL and b"Philox" in lib.tnmc_last_error()
    env = ctypes.c_void_p(0)
    p = _fake_problem((8,), T.COUPLING_PMJ)
    rc = lib.tnmc_run(ctypes.byref(p._c), T.FP32, fake, 1 << 30, 8, 0, (1 << 32) - 1, fake, 0, 0, fake, fake,
                      fake, fake, None, None, 0, None, ctypes.byref(env))
    assert rc == T.TNMC_EINVAL and b"Philox" in lib.tnmc_last_error()


def test_autotune_validation(lib):
    p = _problem((16, 32), (8, 16), (1.0, 0.5))
    assert lib.tnmc_autotune_workspace_bytes(ctypes.byref(p._c), T.FP32, 16, 4) > 0
    assert lib.tnmc_autotune_workspace_bytes(ctypes.byref(p._c), T.FP32, 16, 0) == 0
    out = T._Tuning()
    # no couplings / bad objective: rejected before any device work
    assert lib.tnmc_autotune(ctypes.byref(p._c), T.FP32, 16, 0, 4, None, 0, None, None,
                             ctypes.byref(out)) == T.TNMC_EINVAL
    q = _fake_problem((16, 32), T.COUPLING_GENERAL)
    assert lib.tnmc_autotune(ctypes.byref(q._c), T.FP32, 16, 9, 4, None, 0, None, None,
                             ctypes.byref(out)) == T.TNMC_EINVAL
    assert lib.tnmc_autotune(ctypes.byref(q._c), T.FP32, 16, 0, 4, None, 0, None, None, None) == T.TNMC_EINVAL
