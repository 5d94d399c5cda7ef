"""FP64 reference of the learned-tail network (test infrastructure only).

Plain numpy definitions of the small MLP that predicts a pixel's tail
composite from 9 tail features: its forward pass, loss, gradients (by the
chain rule, written out layer by layer) and the Adam update.  The GPU
kernels implement the same definitions in BF16 MFMA with FP32 accumulation.

Parameter vector (float, length PARAM_COUNT), in this order:
    mu[9], inv_sigma[9]          input standardisation (not trained)
    W1[9][64], b1[64]            x' = (x - mu) * inv_sigma;  z1 = x' W1 + b1
    W2[64][64], b2[64]           h1 = gelu(z1); z2 = h1 W2 + b2
    W3[64][5], b3[5]             h2 = gelu(z2); y = h2 W3 + b3
Outputs: y[0:4] = tail premultiplied RGBA, y[4] = confidence logit.
GELU is the tanh form.  With bf16=True, forward and backward round to BF16
(round to nearest even, after an FP32 rounding) exactly the operands the
matrix-core kernels round: the standardised input, the weights, the hidden
activations and the back-propagated output and hidden gradients that enter
products; biases, pre-activations, GELU and its derivative, bias gradients
and all sums stay in wide precision.  This models the kernels' arithmetic for
a tight comparison; bf16=False is the exact FP64 definition.  Loss per sample:
    (1/4) sum_c (y_c - t_c)^2 + LAMBDA * BCE(sigmoid(y_4), label),
    label = 1 when max_c |y_c - t_c| < conf_tol (default CONF_TOL; no gradient
    through the label),
averaged over the samples.
"""
from __future__ import annotations

import math

import numpy as np

NF, NH, NO = 9, 64, 5
LAMBDA = 0.1
CONF_TOL = 2e-3
OFF = {}
_o = 0
for _name, _n in (("mu", NF), ("inv_sigma", NF), ("W1", NF * NH), ("b1", NH), ("W2", NH * NH), ("b2", NH),
                  ("W3", NH * NO), ("b3", NO)):
    OFF[_name] = (_o, _o + _n)
    _o += _n
PARAM_COUNT = _o
TRAINED = np.ones(PARAM_COUNT, dtype=bool)
TRAINED[: 2 * NF] = False

_C = math.sqrt(2.0 / math.pi)


def bf16(x):
    """Round to BF16 (nearest even) through FP32; returns float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, on):
    return bf16(x) if on else x


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    g = lambda k: p[OFF[k][0]:OFF[k][1]]
    return dict(mu=g("mu"), inv_sigma=g("inv_sigma"), W1=g("W1").reshape(NF, NH), b1=g("b1"),
                W2=g("W2").reshape(NH, NH), b2=g("b2"), W3=g("W3").reshape(NH, NO), b3=g("b3"))


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(_C * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = _C * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * _C * (1.0 + 3 * 0.044715 * x * x)


def forward(p, X, bf16=False):
    """Returns y [n,5] and the intermediates needed by backward."""
    P = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    b = bf16
    xs = _r((X - P["mu"]) * P["inv_sigma"], b)
    z1 = xs @ _r(P["W1"], b) + P["b1"]
    h1 = _r(gelu(z1), b)
    z2 = h1 @ _r(P["W2"], b) + P["b2"]
    h2 = _r(gelu(z2), b)
    y = h2 @ _r(P["W3"], b) + P["b3"]
    return y, dict(xs=xs, z1=z1, h1=h1, z2=z2, h2=h2, bf16=b)


def loss_and_dy(y, T, conf_tol=CONF_TOL):
    """Mean loss and dL/dy for targets T [n,4]; the confidence label is
    1[max_c |y_c - t_c| < conf_tol]."""
    y = np.asarray(y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    n = y.shape[0]
    err = y[:, :4] - T
    label = (np.abs(err).max(axis=1) < conf_tol).astype(np.float64)
    s = 1.0 / (1.0 + np.exp(-y[:, 4]))
    bce = -(label * np.log(np.maximum(s, 1e-300)) + (1 - label) * np.log(np.maximum(1 - s, 1e-300)))
    L = float(np.mean(0.25 * (err ** 2).sum(axis=1) + LAMBDA * bce))
    dy = np.zeros_like(y)
    dy[:, :4] = 0.5 * err / n
    dy[:, 4] = LAMBDA * (s - label) / n
    return L, dy


def backward(p, cache, dy):
    """Gradient of sum(dy * y) with respect to the parameter vector (rounding
    as the forward pass that made `cache`)."""
    P = unpack(p)
    b = cache.get("bf16", False)
    g = np.zeros(PARAM_COUNT)
    put = lambda k, v: g.__setitem__(slice(*OFF[k]), np.asarray(v).ravel())
    dz3 = np.asarray(dy, dtype=np.float64)
    dz3r = _r(dz3, b)
    put("W3", cache["h2"].T @ dz3r)
    put("b3", dz3.sum(axis=0))
    dz2 = (dz3r @ _r(P["W3"], b).T) * gelu_grad(cache["z2"])
    dz2r = _r(dz2, b)
    put("W2", cache["h1"].T @ dz2r)
    put("b2", dz2.sum(axis=0))
    dz1 = (dz2r @ _r(P["W2"], b).T) * gelu_grad(cache["z1"])
    put("W1", cache["xs"].T @ _r(dz1, b))
    put("b1", dz1.sum(axis=0))
    return g


def adam_step(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the trained entries (step counts from 1)."""
    p, m, v = p.copy(), m.copy(), v.copy()
    t = TRAINED
    m[t] = b1 * m[t] + (1 - b1) * g[t]
    v[t] = b2 * v[t] + (1 - b2) * g[t] ** 2
    mh = m[t] / (1 - b1 ** step)
    vh = v[t] / (1 - b2 ** step)
    p[t] -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def init_params(feat_mean, feat_std, seed=0):
    """He-style random initialisation with the given input standardisation."""
    rng = np.random.default_rng(seed)
    p = np.zeros(PARAM_COUNT)
    p[slice(*OFF["mu"])] = feat_mean
    p[slice(*OFF["inv_sigma"])] = 1.0 / np.maximum(np.asarray(feat_std, dtype=np.float64), 1e-6)
    p[slice(*OFF["W1"])] = rng.normal(0, math.sqrt(2.0 / NF), NF * NH)
    p[slice(*OFF["W2"])] = rng.normal(0, math.sqrt(2.0 / NH), NH * NH)
    p[slice(*OFF["W3"])] = rng.normal(0, math.sqrt(1.0 / NH), NH * NO) * 0.1
    return p
