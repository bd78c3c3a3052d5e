"""Batched tensor-network Monte Carlo (TNMC) on MI355X -- Python binding.

A thin ctypes layer over the C ABI in include/tnmc.h.  Functions carry the
same names as the C entry points and only marshal arguments: torch tensors
provide device memory and the current HIP stream; every step of the method
runs in the HIP kernels of libtnmc.so.  If the library is missing the calls
raise -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtnmc.so")

TNMC_OK, TNMC_EINVAL, TNMC_ENOSPACE, TNMC_EHIP, TNMC_ENOTSUP, TNMC_ENUMERIC = 0, -1, -2, -3, -4, -5
COUPLING_GENERAL, COUPLING_PMJ, COUPLING_GRID20 = 0, 1, 2
ALTERNATE_SWEEPS = 1
FORCE_F64_FALLBACK = 2
SHORT_WAITS = 8
FP64, FP32, MIXED_BF16, MIXED_FP16, MIXED_BF16X3 = 0, 1, 2, 3, 4
SCHED_LONGEST_FIRST, SCHED_SHORTEST_FIRST, SCHED_AS_GIVEN = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": MIXED_BF16, "fp16": MIXED_FP16, "bf16x3": MIXED_BF16X3}
CHAIN_BYTES = 48           # sizeof(tnmc_chain)

_lib = None


class TnmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tnmc error {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("batch", c_int32), ("L", POINTER(c_int32)), ("chi", POINTER(c_int32)),
                ("beta", POINTER(c_double)), ("J_h", c_void_p), ("J_v", c_void_p),
                ("off_h", POINTER(c_int64)), ("off_v", POINTER(c_int64)), ("coupling_kind", c_int32),
                ("flags", c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("schedule", c_int32), ("split", c_int32), ("objective_s", c_double),
                ("candidates_s", c_double * 4), ("from_cache", c_int32)]


OBJECTIVES = {"p99": 0, "p50": 1, "mean": 2, "makespan": 3}


class _Mlp(ctypes.Structure):
    _fields_ = [("params", c_void_p)]


MLP_NPARAM = 8385
MLP_LAYOUT = {"W1": (0, (64, 64)), "b1": (4096, (64,)), "W2": (4160, (64, 64)), "b2": (8256, (64,)),
              "W3": (8320, (64,)), "b3": (8384, (1,))}


EXPORTS = ("tnmc_workspace_bytes", "tnmc_workspace_size", "tnmc_build_env", "tnmc_run", "tnmc_sample",
           "tnmc_energy", "tnmc_accept", "tnmc_env_check", "tnmc_overlap", "tnmc_autotune",
           "tnmc_autotune_workspace_bytes",
           "tnmc_free_env", "tnmc_last_error", "tnmc_philox_uniform", "tnmc_env_stats",
           "tnmc_mlp_features", "tnmc_mlp_scratch_floats", "tnmc_mlp_train_step", "tnmc_mlp_forward",
           "tnmc_mlp_train_step_noalloc")


def load(path: str = LIB_PATH):
    """Load libtnmc.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise TnmcError(TNMC_EHIP, f"{path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P = POINTER
    lib.tnmc_workspace_size.argtypes = [P(_Problem), c_int32, c_int32, P(c_size_t)]
    lib.tnmc_workspace_bytes.argtypes = [P(_Problem), c_int32, c_int32]
    lib.tnmc_workspace_bytes.restype = c_size_t
    lib.tnmc_env_check.argtypes = [c_void_p, c_void_p]
    lib.tnmc_autotune_workspace_bytes.argtypes = [P(_Problem), c_int32, c_int32, c_int32]
    lib.tnmc_autotune_workspace_bytes.restype = c_size_t
    lib.tnmc_autotune.argtypes = [P(_Problem), c_int32, c_int32, c_int32, c_int32, c_void_p, c_size_t,
                                  ctypes.c_char_p, c_void_p, P(_Tuning)]
    lib.tnmc_autotune.restype = c_int
    lib.tnmc_overlap.argtypes = [P(_Problem), c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_uint64, c_void_p,
                                 c_void_p]
    lib.tnmc_build_env.argtypes = [P(_Problem), c_int32, c_void_p, c_size_t, c_void_p, P(c_void_p), c_void_p]
    lib.tnmc_run.argtypes = [P(_Problem), c_int32, c_void_p, c_size_t, c_int32, c_uint64, c_uint64, c_void_p,
                             c_uint64, c_uint64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_int32, c_void_p, P(c_void_p)]
    lib.tnmc_sample.argtypes = [c_void_p, c_int32, c_uint64, c_uint64, c_void_p, P(_Mlp), c_void_p,
                                c_void_p, c_void_p, c_void_p]
    lib.tnmc_energy.argtypes = [P(_Problem), c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.tnmc_accept.argtypes = [c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_uint64,
                                c_uint64, c_void_p, c_void_p, c_void_p]
    lib.tnmc_free_env.argtypes = [c_void_p]
    lib.tnmc_free_env.restype = None
    lib.tnmc_last_error.restype = ctypes.c_char_p
    lib.tnmc_philox_uniform.argtypes = [c_uint64, c_void_p, c_uint32, c_uint32, c_uint32, c_int32,
                                        c_void_p, c_void_p]
    lib.tnmc_env_stats.argtypes = [c_void_p]
    lib.tnmc_env_stats.restype = c_void_p
    lib.tnmc_mlp_features.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.tnmc_mlp_scratch_floats.argtypes = [c_int32]
    lib.tnmc_mlp_scratch_floats.restype = c_size_t
    lib.tnmc_mlp_train_step.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                        ctypes.c_float, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.tnmc_mlp_forward.argtypes = [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_void_p]
    lib.tnmc_mlp_train_step_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                                c_void_p, ctypes.c_float, c_int32, c_void_p, c_void_p, c_void_p]
    for name in ("tnmc_workspace_size", "tnmc_build_env", "tnmc_sample", "tnmc_energy", "tnmc_env_check",
                 "tnmc_overlap",
                 "tnmc_accept", "tnmc_philox_uniform", "tnmc_mlp_features", "tnmc_mlp_train_step",
                 "tnmc_mlp_forward", "tnmc_mlp_train_step_noalloc"):
        getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != TNMC_OK:
        raise TnmcError(rc, _lib.tnmc_last_error().decode())


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


class Problem:
    """Host-side problem description; J_h / J_v are device float32 tensors.

    Either uniform: J_h (B, L, L-1), J_v (B, L-1, L) with scalar or per-instance
    chi/beta; or uneven: flat J_h / J_v with per-instance L and offsets.
    coupling_kind is one of COUPLING_GENERAL, COUPLING_PMJ, COUPLING_GRID20;
    flags 0, ALTERNATE_SWEEPS and/or FORCE_F64_FALLBACK.
    """

    def __init__(self, J_h, J_v, L, chi, beta, off_h=None, off_v=None, coupling_kind=COUPLING_GENERAL, flags=0):
        import numpy as np
        self.J_h, self.J_v = J_h, J_v
        B = len(L)
        self.L = np.ascontiguousarray(L, dtype=np.int32)
        self.chi = np.ascontiguousarray(np.broadcast_to(chi, (B,)), dtype=np.int32)
        self.beta = np.ascontiguousarray(np.broadcast_to(beta, (B,)), dtype=np.float64)
        self.off_h = None if off_h is None else np.ascontiguousarray(off_h, dtype=np.int64)
        self.off_v = None if off_v is None else np.ascontiguousarray(off_v, dtype=np.int64)
        self.batch = B
        self.coupling_kind = int(coupling_kind)
        self.flags = int(flags)
        self._c = _Problem(
            B, self.L.ctypes.data_as(POINTER(c_int32)), self.chi.ctypes.data_as(POINTER(c_int32)),
            self.beta.ctypes.data_as(POINTER(c_double)),
            None if J_h is None else J_h.data_ptr(), None if J_v is None else J_v.data_ptr(),
            None if self.off_h is None else self.off_h.ctypes.data_as(POINTER(c_int64)),
            None if self.off_v is None else self.off_v.ctypes.data_as(POINTER(c_int64)), self.coupling_kind,
            self.flags)

    @classmethod
    def uniform(cls, J_h, J_v, chi, beta):
        B, L = J_h.shape[0], J_h.shape[1]
        return cls(J_h, J_v, [L] * B, chi, beta)

    def words(self):
        return [(int(L) + 63) // 64 for L in self.L]

    def spin_words_per_sample(self):
        return sum(int(L) * w for L, w in zip(self.L, self.words()))


def tnmc_workspace_bytes(problem: Problem, precision: int, max_samples: int) -> int:
    """Workspace bytes for the problem (0 on a bad problem; see tnmc_last_error)."""
    return load().tnmc_workspace_bytes(byref(problem._c), precision, max_samples)


def tnmc_workspace_size(problem: Problem, precision: int, max_samples: int) -> int:
    lib = load()
    out = c_size_t(0)
    _check(lib.tnmc_workspace_size(byref(problem._c), precision, max_samples, byref(out)))
    return out.value


class Env:
    def __init__(self, handle, problem, precision, workspace):
        self.handle, self.problem, self.precision, self.workspace = handle, problem, precision, workspace

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.tnmc_free_env(self.handle)
            self.handle = None


def tnmc_build_env(problem: Problem, precision: int, workspace, logz_out=None, stream=None) -> Env:
    """Build every instance's boundary-MPS cache into `workspace` (a uint8
    device tensor of at least tnmc_workspace_size bytes)."""
    lib = load()
    h = c_void_p(0)
    _check(lib.tnmc_build_env(byref(problem._c), precision, _ptr(workspace), workspace.numel(),
                              _stream(stream), byref(h), _ptr(logz_out)))
    return Env(h, problem, precision, workspace)


def tnmc_run(problem: Problem, precision: int, workspace, n_samples: int, sample_seed: int, chain,
             accept_seed: int, spins_out, logq_out, E_out, accepted_out, state_out=None, logz_out=None,
             sample_offset: int = 0, step_offset: int = 0, schedule: int = 0, stream=None) -> Env:
    """Build, sample, score and accept every instance in one persistent
    launch (each instance finishes on its own); schedule is one of
    SCHED_LONGEST_FIRST, SCHED_SHORTEST_FIRST, SCHED_AS_GIVEN.  Returns the
    env."""
    lib = load()
    h = c_void_p(0)
    _check(lib.tnmc_run(byref(problem._c), precision, _ptr(workspace), workspace.numel(), n_samples,
                        sample_seed, sample_offset, _ptr(chain), accept_seed, step_offset, _ptr(spins_out),
                        _ptr(logq_out), _ptr(E_out), _ptr(accepted_out), _ptr(state_out), _ptr(logz_out),
                        schedule, _stream(stream), byref(h)))
    return Env(h, problem, precision, workspace)


def tnmc_sample(env: Env, n_samples: int, seed: int, spins_out, logq_out, sample_offset: int = 0,
                forced_spins=None, mlp=None, logits_out=None, stream=None):
    """mlp: None, or a device float32 tensor of MLP_NPARAM parameters."""
    lib = load()
    m = None
    if mlp is not None:
        m = _Mlp(mlp.data_ptr())
    _check(lib.tnmc_sample(env.handle, n_samples, seed, sample_offset, _ptr(forced_spins),
                           None if m is None else byref(m), _ptr(spins_out), _ptr(logq_out),
                           _ptr(logits_out), _stream(stream)))


def tnmc_energy(problem, n_samples: int, spins, E_out, E_int_out=None, stream=None):
    """problem: a Problem, or an Env (its problem is used).  E_int_out (int32
    (B, N), optional) needs coupling_kind COUPLING_PMJ."""
    lib = load()
    if isinstance(problem, Env):
        problem = problem.problem
    _check(lib.tnmc_energy(byref(problem._c), n_samples, _ptr(spins), _ptr(E_out), _ptr(E_int_out),
                           _stream(stream)))


def tnmc_overlap(problem, n_samples: int, spins_a, state_a, spins_b, state_b, q_out, state_offset: int = 0,
                 stream=None):
    """Replica overlap of two chains' current states after each step (see
    tnmc.h); problem may be an Env."""
    lib = load()
    if isinstance(problem, Env):
        problem = problem.problem
    _check(lib.tnmc_overlap(byref(problem._c), n_samples, _ptr(spins_a), _ptr(state_a), _ptr(spins_b),
                            _ptr(state_b), state_offset, _ptr(q_out), _stream(stream)))


def tnmc_autotune(problem: Problem, precision: int, n_samples: int, objective: str = "p99",
                  replica_scale: int = 4, cache_path=None, stream=None) -> dict:
    """Schedule choice for tnmc_run on this batch (timed on a sub-lattice
    replica in the library, or read from the tuning cache).  Returns a dict
    with schedule, split, objective_s, candidates_s and from_cache."""
    import torch
    lib = load()
    nbytes = lib.tnmc_autotune_workspace_bytes(byref(problem._c), precision, n_samples, replica_scale)
    if nbytes == 0:
        raise TnmcError(TNMC_EINVAL, lib.tnmc_last_error().decode())
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = _Tuning()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib.tnmc_autotune(byref(problem._c), precision, n_samples, OBJECTIVES[objective], replica_scale,
                             _ptr(ws), nbytes, path, _stream(stream), byref(out)))
    return {"schedule": out.schedule, "split": bool(out.split), "objective_s": out.objective_s,
            "candidates_s": list(out.candidates_s), "from_cache": bool(out.from_cache)}


def tnmc_env_check(env: Env, stream=None):
    """Synchronises the stream; raises TnmcError(TNMC_ENUMERIC) if a build
    produced a non-finite log-scale or a Jacobi stopped at its sweep limit."""
    _check(load().tnmc_env_check(env.handle, _stream(stream)))


def tnmc_accept(logq, E, beta, chain, seed: int, step_offset: int, accepted_out, state_out=None,
                stream=None):
    """logq, E: (B, N) float64; beta: (B,) float64; chain: uint8 (B*48,) zero-
    initialised device tensor; accepted_out uint8 (B, N); state_out int64."""
    lib = load()
    B, N = logq.shape
    _check(lib.tnmc_accept(B, N, _ptr(logq), _ptr(E), _ptr(beta), _ptr(chain), seed, step_offset,
                           _ptr(accepted_out), _ptr(state_out), _stream(stream)))


def tnmc_philox_uniform(seed: int, c0, c1: int, c2: int, stream_id: int, out, stream=None):
    lib = load()
    _check(lib.tnmc_philox_uniform(seed, _ptr(c0), c1, c2, stream_id, c0.numel(), _ptr(out),
                                   _stream(stream)))


STATS_PER_INST = 16
STAT_MAXSWEEP, STAT_NONFINITE, STAT_LOGZ_UNDEFINED, STAT_FALLBACK, STAT_PIPE_ERROR = 8, 9, 10, 11, 12


def tnmc_env_stats(env: Env):
    """Per-instance statistics as a host int64 array (B, 16): Jacobi sweeps;
    100 MHz ticks spent in the QR sweeps, the SVD sweeps and the Jacobi
    loops; build start and end ticks; end tick of the first sampling tile
    of the last tnmc_sample call; ticks in the Householder factorisations;
    truncations whose Jacobi reached the sweep limit; non-finite row
    log-scales; 1 if ln Z is undefined (the truncated network's total was
    not positive).  Synchronises the current stream."""
    import numpy as np
    import torch
    addr = load().tnmc_env_stats(env.handle)
    off = addr - env.workspace.data_ptr()
    torch.cuda.current_stream().synchronize()
    n = 8 * STATS_PER_INST * env.problem.batch
    return env.workspace[off:off + n].view(torch.int64).cpu().numpy().reshape(-1, STATS_PER_INST)


def chain_state(chain_bytes):
    """Decode a host copy of the chain array into a list of dicts."""
    import numpy as np
    raw = np.frombuffer(bytes(chain_bytes), dtype=np.uint8).reshape(-1, CHAIN_BYTES)
    out = []
    for row in raw:
        f = np.frombuffer(row[:16].tobytes(), dtype=np.float64)
        i = np.frombuffer(row[16:].tobytes(), dtype=np.int64)
        out.append(dict(cur_logq=f[0], cur_E=f[1], cur_index=int(i[0]), n_acc=int(i[1]),
                        n_trials=int(i[2]), initialised=int(i[3])))
    return out


def tnmc_mlp_features(env: Env, n_samples: int, spins, logits_lo, feat_out, stream=None):
    lib = load()
    _check(lib.tnmc_mlp_features(env.handle, n_samples, _ptr(spins), _ptr(logits_lo), _ptr(feat_out),
                                 _stream(stream)))


def tnmc_mlp_scratch_floats(n_rows: int) -> int:
    return load().tnmc_mlp_scratch_floats(n_rows)


def tnmc_mlp_train_step(params, adam_m, adam_v, feat, logit_lo, target_logit, lr: float, step: int,
                        scratch, grad_out=None, loss_out=None, stream=None):
    lib = load()
    n = logit_lo.numel()
    _check(lib.tnmc_mlp_train_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), n, _ptr(feat), _ptr(logit_lo),
                                   _ptr(target_logit), float(lr), step, _ptr(scratch), _ptr(grad_out),
                                   _ptr(loss_out), _stream(stream)))


MLP_NOALLOC_MAX_ROWS = 16384


def tnmc_mlp_train_step_noalloc(params, adam_m, adam_v, feat, logit_lo, target_logit, lr: float, step: int,
                                grad_out=None, loss_out=None, stream=None):
    """tnmc_mlp_train_step with the library's static per-GPU scratch (at most
    MLP_NOALLOC_MAX_ROWS rows; overlapping calls on one GPU race)."""
    lib = load()
    n = logit_lo.numel()
    _check(lib.tnmc_mlp_train_step_noalloc(_ptr(params), _ptr(adam_m), _ptr(adam_v), n, _ptr(feat),
                                           _ptr(logit_lo), _ptr(target_logit), float(lr), step, _ptr(grad_out),
                                           _ptr(loss_out), _stream(stream)))


def tnmc_mlp_forward(params, feat, d_out, bf16_weights: bool = False, stream=None):
    lib = load()
    _check(lib.tnmc_mlp_forward(_ptr(params), d_out.numel(), _ptr(feat), int(bf16_weights), _ptr(d_out),
                                _stream(stream)))
