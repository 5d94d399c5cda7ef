"""Pins of the learned-tail oracle (network and tail features) on the CPU.

The network reference (oracle/mlp.py) is pinned by central finite
differences of its own loss (backward must be the derivative of forward),
hand-built weight patterns with scalar closed forms (catching transposed
weights and wrong offsets), the erf form of GELU, Adam's closed form under a
constant gradient and the BF16 rounding rule.  The tail features
(orc_frame_tail) are pinned on a column of equal layers whose head, tail,
opacity sums and depth moments have closed forms, and by the associativity
of the "over" operator against the full exact composite.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from oracle import mlp
from tests.test_oracle_pins import column_setup, flat_style


def rand_params(seed=0):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(rng.normal(0, 1, mlp.NF), rng.uniform(0.5, 2.0, mlp.NF), seed=seed)
    p[slice(*mlp.OFF["b1"])] = rng.normal(0, 0.3, mlp.NH)
    p[slice(*mlp.OFF["b2"])] = rng.normal(0, 0.3, mlp.NH)
    p[slice(*mlp.OFF["b3"])] = rng.normal(0, 0.3, mlp.NO)
    p[slice(*mlp.OFF["W3"])] *= 10.0
    return p


def mean_loss(p, X, T):
    y, _ = mlp.forward(p, X)
    return mlp.loss_and_dy(y, T)[0]


def test_param_layout():
    assert mlp.PARAM_COUNT == 18 + 9 * 64 + 64 + 64 * 64 + 64 + 64 * 5 + 5 == 5143
    assert not mlp.TRAINED[:18].any() and mlp.TRAINED[18:].all()


def test_bf16_rounding_rule():
    one = 1.0
    assert mlp.bf16(one) == 1.0
    assert mlp.bf16(1 + 2 ** -8) == 1.0                   # tie, to even
    assert mlp.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6       # tie, to even (up)
    assert mlp.bf16(1 + 2 ** -8 + 2 ** -12) == 1 + 2 ** -7  # above the tie
    assert mlp.bf16(-3.0) == -3.0
    x = np.random.default_rng(1).normal(0, 10, 1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8 * (1 + 1e-6))


def test_gelu_close_to_erf_form():
    xs = np.linspace(-6, 6, 241)
    exact = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    assert np.max(np.abs(mlp.gelu(xs) - exact)) < 5e-4
    assert mlp.gelu(np.array([0.0]))[0] == 0.0


def test_gelu_grad_is_derivative():
    xs = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (mlp.gelu(xs + h) - mlp.gelu(xs - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(xs))) < 1e-8


def test_forward_hand_built_weights():
    """x' = e_0, W1[0][j] = a_j, W2 = I, W3[:, 0] = 1: y_0 = sum_j gelu(gelu(a_j + b1_j) + b2_j)."""
    rng = np.random.default_rng(3)
    p = np.zeros(mlp.PARAM_COUNT)
    mu = rng.normal(0, 1, 9)
    sig = rng.uniform(0.5, 2, 9)
    p[slice(*mlp.OFF["mu"])] = mu
    p[slice(*mlp.OFF["inv_sigma"])] = 1 / sig
    a = rng.normal(0, 1, 64)
    b1 = rng.normal(0, 0.5, 64)
    b2 = rng.normal(0, 0.5, 64)
    W1 = np.zeros((9, 64))
    W1[0] = a
    W1[4, 7] = 100.0  # input 4 is zero after standardisation: must not matter
    p[slice(*mlp.OFF["W1"])] = W1.ravel()
    p[slice(*mlp.OFF["b1"])] = b1
    p[slice(*mlp.OFF["W2"])] = np.eye(64).ravel()
    p[slice(*mlp.OFF["b2"])] = b2
    W3 = np.zeros((64, 5))
    W3[:, 0] = 1.0
    W3[5, 3] = 2.0
    p[slice(*mlp.OFF["W3"])] = W3.ravel()
    p[slice(*mlp.OFF["b3"])] = [0, 0, 0, 0, 0.25]
    x = mu.copy()
    x[0] += sig[0]  # standardised input = e_0
    y, _ = mlp.forward(p, x[None, :])
    g = lambda v: 0.5 * v * (1 + math.tanh(math.sqrt(2 / math.pi) * (v + 0.044715 * v ** 3)))
    h2 = [g(g(a[j] + b1[j]) + b2[j]) for j in range(64)]
    assert y[0, 0] == pytest.approx(sum(h2), rel=1e-12)
    assert y[0, 3] == pytest.approx(2.0 * h2[5], rel=1e-12)
    assert y[0, 1] == 0.0 and y[0, 2] == 0.0
    assert y[0, 4] == 0.25


def test_loss_closed_forms():
    y = np.array([[0.1, 0.2, 0.3, 0.4, 1.5], [0.1, 0.2, 0.3, 0.4, -0.7]])
    T = np.array([[0.1, 0.2, 0.3, 0.4], [0.6, 0.2, 0.3, 0.1]])
    L, dy = mlp.loss_and_dy(y, T)
    l0 = 0.1 * math.log1p(math.exp(-1.5))                       # label 1, no error
    l1 = 0.25 * (0.25 + 0.09) + 0.1 * math.log1p(math.exp(-0.7))  # label 0
    assert L == pytest.approx((l0 + l1) / 2, rel=1e-12)
    s = lambda v: 1 / (1 + math.exp(-v))
    assert dy[0, 4] == pytest.approx(0.1 * (s(1.5) - 1) / 2, rel=1e-12)
    assert dy[1, 4] == pytest.approx(0.1 * s(-0.7) / 2, rel=1e-12)
    assert dy[1, 0] == pytest.approx(0.5 * -0.5 / 2, rel=1e-12)
    assert np.all(dy[0, :4] == 0)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(7)
    p = rand_params(7)
    n = 24
    X = rng.normal(0, 1, (n, 9)) * p[9:18] ** -1 + p[:9]
    y0, _ = mlp.forward(p, X)
    T = rng.uniform(0, 1, (n, 4))
    T[:6] = y0[:6, :4]  # rows with label 1
    L, dy = mlp.loss_and_dy(y0, T)
    _, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, dy)
    assert np.all(g[:18] == 0)
    idx = np.concatenate([rng.choice(np.arange(18, mlp.PARAM_COUNT), 300, replace=False),
                          np.arange(*mlp.OFF["b3"]), np.arange(mlp.OFF["W1"][0], mlp.OFF["W1"][0] + 20)])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mean_loss(pp, X, T) - mean_loss(pm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_model_is_close_to_fp64():
    rng = np.random.default_rng(11)
    p = rand_params(11)
    X = rng.normal(0, 1, (200, 9)) * p[9:18] ** -1 + p[:9]
    y, c = mlp.forward(p, X)
    yb, cb = mlp.forward(p, X, bf16=True)
    err = np.abs(y - yb).max() / np.abs(y).max()
    assert 0 < err < 2e-2
    T = rng.uniform(0, 1, (200, 4))
    _, dy = mlp.loss_and_dy(y, T)
    g = mlp.backward(p, c, dy)
    gb = mlp.backward(p, cb, dy)
    assert 0 < np.linalg.norm(g - gb) / np.linalg.norm(g) < 2e-2


def test_adam_closed_form_constant_gradient():
    rng = np.random.default_rng(5)
    p0 = rng.normal(0, 1, mlp.PARAM_COUNT)
    g = rng.normal(0, 1e-3, mlp.PARAM_COUNT)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    p = p0
    lr, eps = 1e-2, 1e-8
    for t in range(1, 6):
        p, m, v = mlp.adam_step(p, m, v, g, t, lr, eps=eps)
        # with a constant gradient the bias-corrected moments are g and g^2
        step = lr * g / (np.abs(g) + eps)
        assert np.allclose(p[18:], p0[18:] - t * step[18:], rtol=0, atol=1e-12)
        assert np.all(p[:18] == p0[:18])


# ---------------------------------------------------------------- tail features
@pytest.mark.parametrize("n,K,a", [(12, 8, 0.1), (20, 4, 0.05), (6, 3, 0.3)])
def test_tail_column_closed_forms(oracle_lib, n, K, a):
    """n cells stacked along the view axis: n + 1 equal layers at view depth
    w_i = 2 + 0.1 i, whose normalised depths are i / n."""
    orc = oracle_lib
    m, cam = column_setup(n)
    st = flat_style(tf_a_lo=a, tf_a_hi=a)
    far = synth.Hotspot((50.0, 50.0, 50.0), 0.1)
    om = orc.Mesh.from_synth(m)
    W = cam.width
    pix = np.array([(W // 2) * W + W // 2, (W // 2 - 1) * W + W // 2 - 1])
    fr = orc.Frame.from_camera(om, cam, pix)
    w0, w1 = orc.view_depth_range(om.export()["pos_q"], cam.view_proj)
    # (positions are quantised to 2^-16, the camera matrix is FP32)
    assert w0 == pytest.approx(2.0, abs=1e-5) and w1 == pytest.approx(2.0 + 0.1 * n, abs=1e-5)
    head, feat, target, has = fr.tail(far, st, K, w0, w1)
    full = orc.render(m, cam, far, st, pixels=pix)["rgba"]
    c = np.array(st.tf_rgb_lo)
    nt = n + 1 - K
    zi = np.arange(K, n + 1) / n
    for s in range(2):
        assert has[s]
        assert head[s, 3] == pytest.approx(1 - (1 - a) ** K, abs=1e-12)
        assert head[s, :3] == pytest.approx(c * (1 - (1 - a) ** K), abs=1e-12)
        assert target[s, 3] == pytest.approx(1 - (1 - a) ** nt, abs=1e-12)
        # over is associative: head over tail = the full composite
        comp = head[s] + (1 - head[s, 3]) * target[s]
        assert comp == pytest.approx(full[s], abs=1e-12)
        assert feat[s, 0] == pytest.approx(math.log1p(nt), abs=1e-12)
        assert feat[s, 1] == pytest.approx(nt * a, abs=1e-12)
        for k in (1, 2):
            assert feat[s, 1 + k] == pytest.approx(np.mean(zi ** k), abs=5e-5)
        # proxy composite of nt equal layers: alpha 1 - (1 - a)^nt, colour c * alpha
        pa = 1 - (1 - a) ** nt
        assert feat[s, 7] == pytest.approx(pa, abs=1e-12)
        assert feat[s, 4:7] == pytest.approx(c * pa, abs=1e-12)
        assert feat[s, 8] == pytest.approx(K / n, abs=5e-5)


def test_tail_short_lists_have_no_row(oracle_lib):
    orc = oracle_lib
    m, cam = column_setup(4)
    W = cam.width
    pix = np.array([(W // 2) * W + W // 2])
    om = orc.Mesh.from_synth(m)
    fr = orc.Frame.from_camera(om, cam, pix)
    w0, w1 = orc.view_depth_range(om.export()["pos_q"], cam.view_proj)
    head, feat, target, has = fr.tail(synth.Hotspot((50.0, 50.0, 50.0), 0.1), flat_style(), 5, w0, w1)
    assert not has[0] and np.all(feat == 0) and np.all(head == 0)


def test_tail_focus_removes_proxy_opacity(oracle_lib):
    """Proxy opacity carries the focus factor min(d / r, 1)^4: a hotspot
    around the whole column makes every tail proxy opacity (nearly) vanish."""
    orc = oracle_lib
    n, K = 10, 4
    m, cam = column_setup(n)
    W = cam.width
    pix = np.array([(W // 2) * W + W // 2])
    om = orc.Mesh.from_synth(m)
    fr = orc.Frame.from_camera(om, cam, pix)
    w0, w1 = orc.view_depth_range(om.export()["pos_q"], cam.view_proj)
    st = flat_style(tf_a_lo=0.2, tf_a_hi=0.2)
    _, far, _, _ = fr.tail(synth.Hotspot((50.0, 50.0, 50.0), 0.1), st, K, w0, w1)
    _, near, _, _ = fr.tail(synth.Hotspot((0.0, 0.0, -0.5), 100.0), st, K, w0, w1)
    assert far[0, 1] == pytest.approx((n + 1 - K) * 0.2, abs=1e-12)
    assert 0 < near[0, 1] < 1e-6


def test_tail_proxy_composite_is_front_to_back(oracle_lib):
    """Cells of increasing importance along the column give faces of
    different proxy colour and opacity; the proxy composite must be the
    front-to-back one (which differs from that of the reversed order)."""
    orc = oracle_lib
    n, K = 12, 2
    m, cam = column_setup(n)
    W = cam.width
    pix = np.array([(W // 2) * W + W // 2])
    sc = np.arange(n, dtype=np.float32) ** 2  # importance grows towards the back (cell k at z = -0.1 (n - k))
    om = orc.Mesh(m.xyz, m.hex, cell_scalar=sc[::-1].copy())
    ex = om.export()
    fr = orc.Frame.from_camera(om, cam, pix)
    w0, w1 = orc.view_depth_range(ex["pos_q"], cam.view_proj)
    st = flat_style(tf_a_lo=0.1, tf_a_hi=0.7)
    _, feat, _, _ = fr.tail(synth.Hotspot((50.0, 50.0, 50.0), 0.1), st, K, w0, w1)
    zq = ex["pos_q"][:, 2] / 65536.0
    lo, hi = np.array(st.tf_rgb_lo), np.array(st.tf_rgb_hi)
    layers = []
    for i in range(K, n + 1):  # cap face at z = -0.1 i
        f = [f for f in range(om.F) if np.all(np.abs(zq[ex["face_v"][f]] + 0.1 * i) < 1e-4)]
        assert len(f) == 1
        tb = float(np.mean(ex["t_v"][ex["face_v"][f[0]]]))
        layers.append((0.1 + 0.6 * tb, lo + (hi - lo) * tb))
    C, A = np.zeros(3), 0.0
    for al, col in layers:
        C += (1 - A) * al * col
        A += (1 - A) * al
    Cr, Ar = np.zeros(3), 0.0  # the same layers in reversed depth order
    for al, col in layers[::-1]:
        Cr += (1 - Ar) * al * col
        Ar += (1 - Ar) * al
    assert abs(Ar - A) < 1e-12 and np.abs(Cr - C).max() > 1e-2  # the pin discriminates the order
    assert feat[0, 7] == pytest.approx(A, abs=1e-12)
    assert feat[0, 4:7] == pytest.approx(C, abs=1e-12)
