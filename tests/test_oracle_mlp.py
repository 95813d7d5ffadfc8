"""Pins for the oracle's warm-start network: backprop against central finite differences,
Adam's first step against its closed form, and the feature scaling conventions."""
import numpy as np

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(3)
    p["b1"] = rng.normal(size=64) * 0.1
    p["b2"] = rng.normal(size=64) * 0.1
    X = rng.normal(size=(40, 4))
    t = rng.normal(size=40)
    L, g = mlp.loss_and_grad(p, X, t)
    flat = mlp.flatten(p)
    gflat = mlp.flatten(g)
    idx = rng.choice(len(flat), 60, replace=False)
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        Lp, _ = mlp.loss_and_grad(mlp.unflatten(fp), X, t)
        Lm, _ = mlp.loss_and_grad(mlp.unflatten(fm), X, t)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-7 * max(1.0, abs(fd))


def test_adam_first_step_closed_form():
    flat = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    out = mlp.adam_update(flat.copy(), g, m, v, 1, lr=0.01, eps=1e-8)
    # first step: m_hat = g, v_hat = g^2 -> update = lr g / (|g| + eps)
    assert np.allclose(out, flat - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)


def test_features_and_prediction_scaling():
    rng = np.random.default_rng(1)
    e_n, e1, e2, dg = (rng.normal(size=100) * s for s in (3.0, 3.0, 3.0, 1e-12))
    X, s_d, s_g = mlp.features(e_n, e1, e2, dg)
    for c in range(4):
        assert np.isclose(np.sqrt(np.mean(X[:, c] ** 2)), 1.0) or c == 2
    # the quadratic extrapolation's increment is linear in the inputs, in units of s_d
    e_n, e1, e2 = 1.0 + 0.01 * rng.normal(size=(3, 100)).cumsum(axis=0)
    X, s_d, _ = mlp.features(e_n, e1, e2, dg)
    assert np.allclose(s_d * (2.0 * X[:, 1] - X[:, 2]), 2.0 * e_n - 3.0 * e1 + e2, rtol=1e-12, atol=1e-15)
    X0, s0, g0 = mlp.features(np.zeros(5), np.zeros(5), np.zeros(5), np.zeros(5))
    assert s0 == 1.0 and g0 == 1.0 and not np.any(X0)
    assert mlp.N_PARAMS == 64 * 4 + 64 + 64 * 64 + 64 + 64 + 1
