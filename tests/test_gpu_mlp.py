"""GPU parity of the learned proposal correction against the float64 oracle,
and what the trained network gains over the plain proposal.

Tolerances: float32 kernels against float64 -- gradients within 2e-4 of
the largest gradient entry, Adam parameters within 1e-6, forward within
1e-4 (float32 weights) or 2e-2 relative with cosine >= 0.999 (bfloat16
weights); features bit-exact (they are copies); the sampler's corrected
logits within 2e-4 of TN logit + the float64 network with the same bfloat16
weights (its products take the activations as hi + lo bfloat16 pairs, about
16 significand bits, with float32 accumulation).
"""
import numpy as np
import pytest

import workloads
from oracle import bmps, mlp, sampler

pytestmark = pytest.mark.gpu


def _params_np(P):
    v = P.detach().cpu().numpy().astype(np.float64)
    return {"W1": v[0:4096].reshape(64, 64), "b1": v[4096:4160], "W2": v[4160:8256].reshape(64, 64),
            "b2": v[8256:8320], "W3": v[8320:8384], "b3": v[8384:8385]}


def _rand_params(torch, seed, out_scale=0.5):
    rng = np.random.default_rng(seed)
    v = rng.uniform(-0.3, 0.3, 8385).astype(np.float32)
    v[8320:8385] *= out_scale / 0.3
    return torch.as_tensor(v).cuda()


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (n, 64)).astype(np.float32)
    x[:, 53:] = 0
    lo = rng.normal(0, 3, n).astype(np.float32)
    tg = (lo + rng.normal(0, 0.7, n)).astype(np.float32)
    return x, lo, tg


def test_gradient_and_adam_match_oracle(tnmc):
    import torch
    import tnmc_gpu as G
    G.say("mlp gradient + adam, 1000 rows (16 groups, the last ragged)")
    P = _rand_params(torch, 1)
    x, lo, tg = _rows(1000, 2)
    xt, lot, tgt = (torch.as_tensor(a).cuda() for a in (x, lo, tg))
    scratch = torch.zeros(tnmc.tnmc_mlp_scratch_floats(1000), dtype=torch.float32, device="cuda")
    grad = torch.zeros(8385, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    tnmc.tnmc_mlp_train_step(P, None, None, xt, lot, tgt, 0.0, 0, scratch, grad_out=grad, loss_out=loss)
    torch.cuda.synchronize()
    p = _params_np(P)
    want = mlp.backward(p, x.astype(np.float64), lo.astype(np.float64), tg.astype(np.float64))
    flat = np.concatenate([want[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    got = grad.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - flat)) < 2e-4 * np.max(np.abs(flat))
    assert abs(loss.item() - mlp.loss(p, x.astype(np.float64), lo, tg)) < 1e-5
    # one Adam step against the oracle's
    m = torch.zeros(8385, dtype=torch.float32, device="cuda")
    v = torch.zeros_like(m)
    tnmc.tnmc_mlp_train_step(P, m, v, xt, lot, tgt, 1e-3, 1, scratch)
    torch.cuda.synchronize()
    mo = {k: np.zeros_like(a) for k, a in p.items()}
    vo = {k: np.zeros_like(a) for k, a in p.items()}
    mlp.adam_step(p, want, mo, vo, 1, lr=1e-3)
    newp = _params_np(P)
    for k in p:
        assert np.max(np.abs(newp[k] - p[k])) < 1e-6


def test_forward_matches_oracle(tnmc):
    import torch
    P = _rand_params(torch, 3)
    x, _, _ = _rows(700, 4)
    d = torch.zeros(700, dtype=torch.float32, device="cuda")
    tnmc.tnmc_mlp_forward(P, torch.as_tensor(x).cuda(), d)
    torch.cuda.synchronize()
    want, _ = mlp.forward(_params_np(P), x.astype(np.float64))
    assert np.max(np.abs(d.cpu().numpy() - want)) < 1e-4
    tnmc.tnmc_mlp_forward(P, torch.as_tensor(x).cuda(), d, bf16_weights=True)
    torch.cuda.synchronize()
    got = d.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - want) < 2e-2 * np.linalg.norm(want)
    assert got @ want / (np.linalg.norm(got) * np.linalg.norm(want)) > 0.999


@pytest.mark.parametrize("L,n", [(12, 24), (70, 24), (12, 300)])
def test_features_and_corrected_logits(tnmc, L, n):
    """Features of GPU draws equal the oracle's; with a random network the
    sampler's corrected logits equal TN logit + oracle MLP (bf16 weights).
    At 70 x 70 the 5 x 5 window crosses the 64-column words of the packed
    spins; 300 samples take two tiles of 256, the second mostly idle."""
    import torch
    import tnmc_gpu as G
    chi, beta = 8, 1.0
    Js = [workloads.instance(L, "gauss", 60, i) for i in range(2)]
    G.say(f"mlp features + corrected logits, 2 x {L}x{L} chi 8, {n} samples")
    run = G.Run(Js, chi, beta, tnmc.FP32, max_samples=n)
    P = _rand_params(torch, 5, out_scale=0.2)
    spins = torch.zeros(run.words(n), dtype=torch.int64, device="cuda")
    logq = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    lg = torch.zeros(2 * n * L * L, dtype=torch.float32, device="cuda")
    tnmc.tnmc_sample(run.env, n, 9, spins, logq, mlp=P, logits_out=lg)
    # the TN logits of the same configurations (plain proposal, scored)
    lg_tn = torch.zeros_like(lg)
    tnmc.tnmc_sample(run.env, n, 9, spins.clone(), logq.clone(), forced_spins=spins, logits_out=lg_tn)
    feat = torch.zeros((2 * n * L * L, 64), dtype=torch.float32, device="cuda")
    tnmc.tnmc_mlp_features(run.env, n, spins, lg_tn, feat)
    torch.cuda.synchronize()
    sp = G.unpack(spins.cpu().numpy(), run.Ls, n)
    f = feat.cpu().numpy().reshape(2, n, L, L, 64)
    ltn = lg_tn.cpu().numpy().reshape(2, n, L, L)
    got = lg.cpu().numpy().reshape(2, n, L, L)
    pb = _params_np(P)
    pb = {k: np.asarray(torch.as_tensor(a).to(torch.bfloat16).to(torch.float64)) for k, a in pb.items()}
    for i, (jh, jv) in enumerate(Js):
        sites = [(0, 0), (0, 5), (3, 0), (5, 7), (11, 11), (7, 1)]
        if L > 64:
            sites += [(2, 62), (3, 63), (4, 64), (5, 65), (6, 66), (69, 69), (1, 64), (68, 2)]
        for (r, c) in sites:
            x = mlp.features(sp[i], jh, jv, ltn[i, :, r, c], r, c)
            assert np.array_equal(f[i, :, r, c].astype(np.float64), x.astype(np.float32).astype(np.float64))
            d, _ = mlp.forward(pb, x)
            assert np.max(np.abs(got[i, :, r, c] - (ltn[i, :, r, c] + d))) < 2e-4


def test_zero_network_is_the_plain_proposal(tnmc):
    import torch
    import tnmc_gpu as G
    L, chi, n = 10, 8, 40
    Js = [workloads.instance(L, "pmj", 61, i) for i in range(3)]
    run = G.Run(Js, chi, 1.0, tnmc.FP32, max_samples=n)
    P = _rand_params(torch, 6)
    P[8320:8385] = 0.0          # output layer zero: d == 0 exactly
    out = []
    for m in (None, P):
        spins = torch.zeros(run.words(n), dtype=torch.int64, device="cuda")
        logq = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        tnmc.tnmc_sample(run.env, n, 17, spins, logq, mlp=m)
        torch.cuda.synchronize()
        out.append((spins.cpu().numpy(), logq.cpu().numpy()))
    # both sample on the matrix cores with the same products and the
    # network's output is exactly zero: identical draws, log q equal up to
    # the rounding of the float64 scalar work in two compiled kernels
    assert np.array_equal(out[0][0], out[1][0])
    assert np.max(np.abs(out[0][1] - out[1][1]) / np.abs(out[0][1])) < 1e-12


def test_selection_falls_back_to_the_plain_proposal(tnmc):
    """The acceptance-based selection keeps a network only on a significant paired win:
    an untrained network with a large random output (a correction that can
    only hurt) is rejected, and the plain proposal's acceptances are what the
    caller then samples with."""
    import torch
    import tnmc_gpu as G
    from paper_2509_19006_amd import learned
    L, beta, chi = 16, 1.0, 4
    val_J = [workloads.instance(L, "gauss", 72, i) for i in range(8)]
    G.say("learned correction: the selection rejects a harmful network")
    P = _rand_params(torch, 9, out_scale=3.0)
    chosen, a0, a1 = learned.select(val_J, chi, beta, P, n_samples=128, seed=12)
    G.say(f"  acceptance plain {a0.mean():.4f}, with the random network {a1.mean():.4f}")
    assert chosen is None
    assert a1.mean() < a0.mean()


@pytest.mark.xfail(strict=False, reason=(
    "no measured gain yet: at 32x32, beta 1, chi 2 -> 16 the trained correction lowered the held-out "
    "acceptance (0.2412 plain, 0.2284 with the network, one-sided p 0.82); at 1024x1024 the training loss stayed flat "
    "(0.2794 -> 0.2797) -- the 5x5 window does not see what the truncation gets wrong"))
def test_learned_proposal_gains_on_held_out_disorders(tnmc):
    """Train on chi 16 conditionals of separately seeded disorders, then
    require a paired acceptance gain of the corrected chi 2 proposal over
    the plain one on 16 held-out disorders (one-sided Wilcoxon p < 0.01)."""
    import tnmc_gpu as G
    from scipy import stats
    from paper_2509_19006_amd import learned
    L, beta, lo_chi, hi_chi = 32, 1.0, 2, 16
    train_J = [workloads.instance(L, "gauss", 70, i) for i in range(16)]
    val_J = [workloads.instance(L, "gauss", 71, i) for i in range(16)]
    G.say("learned correction: data (16 disorders x 32 draws at chi 16), training, judging")
    feat, lo, tgt = learned.make_training_data(train_J, lo_chi, hi_chi, beta, 32, seed=3)
    P, losses = learned.train(feat, lo, tgt, steps=400, batch=4096, lr=1e-3, seed=1, log=G.say)
    assert all(np.isfinite(l) for _, l in losses)
    _, a0, a1 = learned.select(val_J, lo_chi, beta, P, n_samples=256, seed=11)
    d = a1 - a0
    pval = stats.wilcoxon(d, alternative="greater").pvalue if np.any(d != 0) else 1.0
    G.say(f"  acceptance plain {a0.mean():.4f}, with network {a1.mean():.4f}, one-sided p {pval:.3g}")
    assert 0.0 < a0.mean() < 1.0
    assert d.mean() > 0 and pval < 0.01
