"""Learned proposal correction: a small MLP on local features (oracle side).

Test infrastructure only: nothing in the product path imports this module.

Not part of the paper; it refines the proposal q of section 2.3, whose
Metropolis step (Eq. 10) keeps sampling exact whatever q is, provided q
covers the support of P.  Per site (r, c) of a configuration the network
sees 64 features:

*  0..19  horizontal couplings J_h[r+dr][c+dc], dr = -2..2, dc = -2..1
* 20..39  vertical couplings J_v[r+dr][c+dc], dr = -2..1, dc = -2..2
* 40..49  spins of rows r-2, r-1 at columns c-2..c+2 (+-1)
* 50..51  spins of row r at columns c-2, c-1 (already sampled)
* 52      the low-chi TN logit, clipped to [-30, 30] and divided by 8
* 53..63  zero
(zero wherever the window leaves the lattice), and outputs a logit
correction d: the corrected conditional is sigmoid(logit + d).

Layers: h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), d = W3 . h2 + b3,
widths 64/64/1.  Loss per site: cross-entropy of the corrected conditional
against a soft target p* = sigmoid(target logit) (the conditional of the
same configuration under a high-chi cache).  Optimiser: Adam (Kingma & Ba,
2015) with bias correction.

Pins (tests/test_oracle_mlp.py): gradients against central finite
differences; a zero last layer leaves every logit unchanged; Adam's first
step with the default moments equals lr * g / (|g| + eps) exactly (the bias
correction undoes the moment decay) and a second step worked out by hand;
training reaches the entropy floor of the targets.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 64, 64


def features(spins, J_h, J_v, logit_lo, r, c):
    """Feature vector(s) of site (r, c).

    spins: (n, L, L) in {-1,+1} (only rows < r and row r left of c are read);
    logit_lo: (n,) low-chi logits at (r, c).  Returns (n, 64) float64.
    """
    spins = np.asarray(spins)
    n, L, _ = spins.shape
    x = np.zeros((n, N_IN))
    k = 0
    for dr in range(-2, 3):
        for dc in range(-2, 2):
            rr, cc = r + dr, c + dc
            if 0 <= rr < L and 0 <= cc < L - 1:
                x[:, k] = J_h[rr, cc]
            k += 1
    for dr in range(-2, 2):
        for dc in range(-2, 3):
            rr, cc = r + dr, c + dc
            if 0 <= rr < L - 1 and 0 <= cc < L:
                x[:, k] = J_v[rr, cc]
            k += 1
    for dr in (-2, -1):
        for dc in range(-2, 3):
            rr, cc = r + dr, c + dc
            if 0 <= rr and 0 <= cc < L:
                x[:, k] = spins[:, rr, cc]
            k += 1
    for dc in (-2, -1):
        cc = c + dc
        if cc >= 0:
            x[:, k] = spins[:, r, cc]
        k += 1
    x[:, k] = np.clip(np.asarray(logit_lo, dtype=np.float64), -30.0, 30.0) / 8.0
    return x


def init_params(seed=0, scale_out=0.0):
    """Glorot-uniform hidden layers; the output layer starts at scale_out
    (0 = the network starts as the identity correction)."""
    rng = np.random.default_rng(seed)
    lim = np.sqrt(6.0 / (N_IN + N_H))
    return {
        "W1": rng.uniform(-lim, lim, (N_H, N_IN)), "b1": np.zeros(N_H),
        "W2": rng.uniform(-lim, lim, (N_H, N_H)), "b2": np.zeros(N_H),
        "W3": rng.uniform(-1, 1, N_H) * scale_out, "b3": np.zeros(1),
    }


def forward(p, x):
    """Returns (d (n,), cache for backward)."""
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(a2)
    d = h2 @ p["W3"] + p["b3"][0]
    return d, (x, h1, h2)


def _sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss(p, x, logit_lo, target_logit):
    """Mean soft-target cross-entropy over the batch."""
    d, _ = forward(p, x)
    z = np.asarray(logit_lo) + d
    t = _sigmoid(np.asarray(target_logit))
    # -[t log s(z) + (1-t) log s(-z)] = softplus(z) - t z
    return float(np.mean(np.logaddexp(0.0, z) - t * z))


def backward(p, x, logit_lo, target_logit):
    """Gradient of `loss` with respect to every parameter (dict)."""
    n = x.shape[0]
    d, (x, h1, h2) = forward(p, x)
    z = np.asarray(logit_lo) + d
    g_d = (_sigmoid(z) - _sigmoid(np.asarray(target_logit))) / n      # dL/dd
    gW3 = h2.T @ g_d
    gb3 = np.array([g_d.sum()])
    g_h2 = np.outer(g_d, p["W3"])
    g_a2 = g_h2 * (1.0 - h2 ** 2)
    gW2 = g_a2.T @ h1
    gb2 = g_a2.sum(axis=0)
    g_h1 = g_a2 @ p["W2"]
    g_a1 = g_h1 * (1.0 - h1 ** 2)
    gW1 = g_a1.T @ x
    gb1 = g_a1.sum(axis=0)
    return {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3}


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; `step` counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
