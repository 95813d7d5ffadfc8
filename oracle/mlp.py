"""Oracle: the per-edge warm-start network in float64 (forward, backward, Adam).

Not from the paper (which has no learned part): a 3-layer perceptron 4 -> 64 -> 64 -> 1
with ReLU, applied to every interior edge independently.  Inputs per edge:
  [e^n / s_e, (e^n - e^{n-1}) / s_d, (e^{n-1} - e^{n-2}) / s_d, dG^{n+1} / s_g],
s_e = RMS of e^n, s_d = RMS of e^n - e^{n-1} and s_g = RMS of dG^{n+1} over interior
edges (each replaced by 1 when zero).  The differences are formed in FP64 before the
inputs are rounded to BF16: successive fields differ by a few per cent, which BF16's
0.4 % rounding of the raw fields would turn into rough per-edge noise.  The output y
predicts the increment in units of s_d: the warm start is x0 = e^n + theta s_d y with
theta the energy-optimal step along s_d y (line-step form) or x0 = e^n + s_d y (direct
form).  Loss: mean squared error of y against (e^{n+1} - e^n) / s_d; a step where that
target's RMS exceeds 10 (the history near zero, as after a neutral start) is not used
for training.

Parameter order and shapes (also the flat layout): W1 [64,4], b1 [64], W2 [64,64],
b2 [64], W3 [1,64], b3 [1].
"""
from __future__ import annotations

import numpy as np

SHAPES = [("W1", (64, 4)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (1, 64)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def init_params(seed):
    """He-uniform weights, zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            fan_in = shp[1]
            lim = np.sqrt(6.0 / fan_in)
            p[name] = g.uniform(-lim, lim, size=shp)
        else:
            p[name] = np.zeros(shp)
    p["W3"] *= 0.1
    return p


def rms_or_one(v):
    s = float(np.sqrt(np.mean(np.asarray(v, dtype=np.float64) ** 2))) if len(v) else 0.0
    return s if s > 0.0 else 1.0


def features(e_n, e_nm1, e_nm2, dG_new):
    """Inputs [n, 4], the increments' unit s_d and s_g."""
    d1, d2 = e_n - e_nm1, e_nm1 - e_nm2
    s_e, s_d, s_g = rms_or_one(e_n), rms_or_one(d1), rms_or_one(dG_new)
    X = np.stack([e_n / s_e, d1 / s_d, d2 / s_d, dG_new / s_g], axis=1)
    return X, s_d, s_g


def forward(p, X):
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ p["W3"].T + p["b3"])[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(p, X, target):
    """L = mean((y - target)^2) and dL/dparams (dict)."""
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n = X.shape[0]
    r = y - target
    L = float(np.mean(r * r))
    dy = (2.0 / n) * r[:, None]                     # [n,1]
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dh2 = dy @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return L, g


def adam_update(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on flat arrays; step counts from 1.  In place."""
    m *= beta1
    m += (1.0 - beta1) * grad
    v *= beta2
    v += (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    flat -= lr * mhat / (np.sqrt(vhat) + eps)
    return flat
