"""Learned proposal correction: data generation, training and evaluation.

Orchestration only -- every numerical step runs in the library's kernels
through the C ABI (tnmc_sample, tnmc_mlp_features, tnmc_mlp_train_step);
torch provides device buffers, index permutations for minibatches and the
parameter initialisation.

Training data are conditionals the method itself computes: configurations
drawn from a high-chi cache, their per-site logits under that cache (the
targets) and, scored on the same configurations, the logits of the low-chi
cache the correction will be applied to (inputs).  The exact Metropolis step
makes any correction safe: a poor network lowers the acceptance rate, never
the correctness; evaluate() compares acceptance with and without it, and
callers keep the plain proposal when the network does not help.
"""
from __future__ import annotations

import math

import numpy as np

from . import (FP32, MLP_NPARAM, Problem, tnmc_build_env, tnmc_mlp_features, tnmc_mlp_scratch_floats,
               tnmc_mlp_train_step, tnmc_sample, tnmc_workspace_size, tnmc_energy, tnmc_accept, CHAIN_BYTES,
               chain_state)


def _env(torch, jh, jv, Ls, chi, beta, n):
    p = Problem(jh, jv, Ls, chi, beta)
    ws = torch.zeros(tnmc_workspace_size(p, FP32, n), dtype=torch.uint8, device="cuda")
    return tnmc_build_env(p, FP32, ws), p


def _flat(torch, Js):
    jh = torch.as_tensor(np.concatenate([np.asarray(a, np.float32).ravel() for a, _ in Js])).cuda()
    jv = torch.as_tensor(np.concatenate([np.asarray(b, np.float32).ravel() for _, b in Js])).cuda()
    return jh, jv, [int(a.shape[0]) for a, _ in Js]


def make_training_data(Js, chi_lo: int, chi_hi: int, beta: float, n_samples: int, seed: int = 1,
                       flip: bool = True):
    """Returns device tensors (features (rows, 64), logit_lo (rows,), target
    logit (rows,)) over every site of n_samples high-chi draws per instance.

    With flip, every row also appears spin-flipped: with no field the flipped
    configuration is equally probable and its conditionals are the mirrored
    ones, so the spin features (slots 40..51), the logit feature (slot 52)
    and both logits change sign while the couplings stay."""
    import torch
    jh, jv, Ls = _flat(torch, Js)
    sites = n_samples * sum(L * L for L in Ls)
    env_hi, p = _env(torch, jh, jv, Ls, chi_hi, beta, n_samples)
    spins = torch.zeros(n_samples * p.spin_words_per_sample(), dtype=torch.int64, device="cuda")
    logq = torch.zeros((len(Ls), n_samples), dtype=torch.float64, device="cuda")
    tgt = torch.zeros(sites, dtype=torch.float32, device="cuda")
    tnmc_sample(env_hi, n_samples, seed, spins, logq, logits_out=tgt)
    env_lo, _ = _env(torch, jh, jv, Ls, chi_lo, beta, n_samples)
    lo = torch.zeros(sites, dtype=torch.float32, device="cuda")
    tnmc_sample(env_lo, n_samples, seed, spins, logq, forced_spins=spins, logits_out=lo)
    feat = torch.zeros((sites, 64), dtype=torch.float32, device="cuda")
    tnmc_mlp_features(env_lo, n_samples, spins, lo, feat)
    torch.cuda.synchronize()
    # sites where either logit is infinite carry no usable target
    ok = torch.isfinite(lo) & torch.isfinite(tgt)
    feat, lo, tgt = feat[ok], lo[ok], tgt[ok]
    if flip:
        sign = torch.ones(64, dtype=torch.float32, device="cuda")
        sign[40:53] = -1.0
        feat = torch.cat([feat, feat * sign])
        lo = torch.cat([lo, -lo])
        tgt = torch.cat([tgt, -tgt])
    return feat.contiguous(), lo.contiguous(), tgt.contiguous()


def init_params(seed: int = 0):
    """Glorot-uniform hidden layers, zero output layer (starts as no correction)."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    p = torch.zeros(MLP_NPARAM, dtype=torch.float32)
    lim = math.sqrt(6.0 / 128.0)
    p[0:4096] = (torch.rand(4096, generator=g) * 2 - 1) * lim
    p[4160:8256] = (torch.rand(4096, generator=g) * 2 - 1) * lim
    return p.cuda()


def train(feat, lo, tgt, steps: int = 600, batch: int = 4096, lr: float = 2e-3, seed: int = 0,
          params=None, log=None):
    """Adam on minibatches of a once-permuted dataset; returns (params, losses)."""
    import torch
    n = lo.numel()
    perm = torch.randperm(n, generator=torch.Generator(device="cpu").manual_seed(seed)).cuda()
    feat, lo, tgt = feat[perm].contiguous(), lo[perm].contiguous(), tgt[perm].contiguous()
    P = init_params(seed) if params is None else params.clone()
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    b = min(batch, n)
    scratch = torch.zeros(tnmc_mlp_scratch_floats(b), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    nb = n // b
    for s in range(1, steps + 1):
        k = (s - 1) % nb
        sl = slice(k * b, (k + 1) * b)
        tnmc_mlp_train_step(P, m, v, feat[sl], lo[sl], tgt[sl], lr, s, scratch, loss_out=loss)
        if s % 50 == 0 or s == steps:
            losses.append((s, float(loss.item())))
            if log:
                log(f"    mlp step {s}: loss {losses[-1][1]:.5f}")
    return P, losses


def acceptance(Js, chi: int, beta: float, n_samples: int, seed: int, mlp=None):
    """Per-instance Metropolis acceptance of the chi proposal (with or
    without the correction) over n_samples draws."""
    import torch
    jh, jv, Ls = _flat(torch, Js)
    env, p = _env(torch, jh, jv, Ls, chi, beta, n_samples)
    B = len(Ls)
    spins = torch.zeros(n_samples * p.spin_words_per_sample(), dtype=torch.int64, device="cuda")
    logq = torch.zeros((B, n_samples), dtype=torch.float64, device="cuda")
    E = torch.zeros((B, n_samples), dtype=torch.float64, device="cuda")
    tnmc_sample(env, n_samples, seed, spins, logq, mlp=mlp)
    tnmc_energy(env, n_samples, spins, E)
    chain = torch.zeros(B * CHAIN_BYTES, dtype=torch.uint8, device="cuda")
    acc = torch.zeros((B, n_samples), dtype=torch.uint8, device="cuda")
    tnmc_accept(logq, E, torch.full((B,), float(beta), dtype=torch.float64, device="cuda"), chain, seed, 0, acc)
    st = chain_state(chain.cpu().numpy())
    return np.array([s["n_acc"] / max(1, s["n_trials"]) for s in st])


def select(Js_val, chi: int, beta: float, mlp_params, n_samples: int = 256, seed: int = 11,
           p_max: float = 0.05):
    """Select the proposal by acceptance on validation disorders.

    Returns (chosen params or None, plain acceptances, learned acceptances):
    the network is kept only if its acceptance beats the plain proposal's,
    paired over disorders, with one-sided Wilcoxon p < p_max; otherwise the
    plain TN proposal is the fallback (None)."""
    from scipy import stats
    a0 = acceptance(Js_val, chi, beta, n_samples, seed)
    a1 = acceptance(Js_val, chi, beta, n_samples, seed, mlp=mlp_params)
    d = a1 - a0
    better = d.mean() > 0 and np.any(d != 0) and stats.wilcoxon(d, alternative="greater").pvalue < p_max
    return (mlp_params if better else None), a0, a1
