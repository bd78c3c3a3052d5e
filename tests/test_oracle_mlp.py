"""Pins for the oracle MLP of the learned proposal correction."""
import numpy as np

import workloads
from oracle import mlp


def _batch(n=40, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (n, mlp.N_IN))
    x[:, 53:] = 0
    lo = rng.normal(0, 3, n)
    tgt = lo + rng.normal(0, 0.5, n)
    return x, lo, tgt


def test_gradients_match_finite_differences():
    p = mlp.init_params(1, scale_out=0.3)
    x, lo, tgt = _batch()
    g = mlp.backward(p, x, lo, tgt)
    rng = np.random.default_rng(2)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(p, x, lo, tgt)
            flat[idx] = old - h
            lm = mlp.loss(p, x, lo, tgt)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) < 1e-7 + 1e-5 * abs(fd), (k, idx)


def test_zero_output_layer_is_identity():
    p = mlp.init_params(3, scale_out=0.0)
    x, lo, _ = _batch()
    d, _ = mlp.forward(p, x)
    assert np.all(d == 0.0)


def test_loss_minimum_at_target():
    """With d = 0 the loss is minimal in the logit exactly when logit = target."""
    p = mlp.init_params(4, scale_out=0.0)
    x, _, tgt = _batch(8)
    base = mlp.loss(p, x, tgt, tgt)
    for eps in (1e-3, -1e-3, 0.5):
        assert mlp.loss(p, x, tgt + eps, tgt) > base


def test_adam_without_moments_is_sign_descent():
    """b1 = b2 = 0 makes Adam's step lr * g / (|g| + eps) (Kingma & Ba, Alg. 1)."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    mlp.adam_step(p, g, m, v, step=1, lr=0.1, b1=0.0, b2=0.0, eps=1e-8)
    want = np.array([1.0, -2.0, 3.0]) - 0.1 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], want, rtol=0, atol=1e-12)


def test_training_reduces_loss():
    p = mlp.init_params(5, scale_out=0.0)
    x, lo, tgt = _batch(256, 6)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(w) for k, w in p.items()}
    t = 0.5 * (1 + np.tanh(0.5 * tgt))
    floor = np.mean(-(t * np.log(t) + (1 - t) * np.log(1 - t)))   # entropy of the targets
    l0 = mlp.loss(p, x, lo, tgt)
    for s in range(1, 201):
        mlp.adam_step(p, mlp.backward(p, x, lo, tgt), m, v, s, lr=3e-3)
    assert mlp.loss(p, x, lo, tgt) - floor < 0.1 * (l0 - floor)


def test_features_window():
    L = 7
    jh, jv = workloads.instance(L, "gauss", 9, 0)
    s = workloads.random_spins(2, L, 1)
    x = mlp.features(s, jh, jv, np.array([4.0, -80.0]), 0, 0)
    # corner site: only bonds and spins inside the lattice survive
    assert x[0, 0 * 4 + 2] == 0 and x[0, 2 * 4 + 2] == jh[0, 0] and x[0, 2 * 4 + 3] == jh[0, 1]
    assert x[0, 20 + 2 * 5 + 2] == jv[0, 0] and np.all(x[:, 40:52] == 0)
    assert x[0, 52] == 0.5 and x[1, 52] == -30 / 8
    x = mlp.features(s, jh, jv, np.zeros(2), 3, 4)
    assert np.array_equal(x[:, 40:45], s[:, 1, 2:7]) and np.array_equal(x[:, 50:52], s[:, 3, 2:4])
    assert np.all(x[:, 53:] == 0)


def test_adam_first_step_is_bias_corrected_sign_step():
    """With the default b1, b2 the bias-corrected first moments equal g and
    g**2 exactly, so step 1 moves every weight by lr * g / (|g| + eps)
    (Kingma & Ba, Alg. 1) -- a missing or wrong correction changes it by
    factors of 10 (1 - b1) or 30 (sqrt(1 - b2))."""
    p = {"w": np.array([0.25, -1.5, 2.0, 0.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3, 2.0])}
    m = {"w": np.zeros(4)}
    v = {"w": np.zeros(4)}
    mlp.adam_step(p, g, m, v, step=1, lr=0.01)
    want = np.array([0.25, -1.5, 2.0, 0.0]) - 0.01 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], want, rtol=0, atol=1e-15)


def test_adam_second_step_by_hand():
    """Step 2 with gradients g1 = 1, g2 = 3 on one weight, the moments and
    the update worked out by hand from Kingma & Ba's Algorithm 1."""
    p = {"w": np.array([1.0])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    lr, b1, b2, eps = 0.1, 0.9, 0.999, 1e-8
    mlp.adam_step(p, {"w": np.array([1.0])}, m, v, 1, lr)
    mlp.adam_step(p, {"w": np.array([3.0])}, m, v, 2, lr)
    # m2 = 0.9 * 0.1 + 0.1 * 3 = 0.39;  v2 = 0.999 * 0.001 + 0.001 * 9 = 0.009999
    # mh = 0.39 / (1 - 0.81) = 2.0526315789...;  vh = 0.009999 / (1 - 0.998001) = 5.0020010005...
    m2, v2 = 0.39, 0.009999
    mh, vh = m2 / 0.19, v2 / 0.001999
    want = 1.0 - lr / (1.0 + eps) - lr * mh / (np.sqrt(vh) + eps)
    assert abs(m["w"][0] - m2) < 1e-15 and abs(v["w"][0] - v2) < 1e-15
    assert abs(p["w"][0] - want) < 1e-14
    assert abs(p["w"][0] - 0.8082219) < 1e-6
