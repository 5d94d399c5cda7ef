"""Pins of the oracle's approximate order-independent resolves (multi-layer
alpha blending, moment-based transparency) on the CPU.

Columns of cap faces seen head-on give pixels whose fragments have known
depth order, known primitive (triangle id) order and per-layer colour and
opacity in closed form (no edges, far hotspot: opacity alpha_TF(t),
colour TF(t) with t the layer's corner importance).  The pins: MLAB with at
least as many layers as fragments is the exact blend; its opacity is exact
for any k; with a non-monotone arrival order and few layers it blends in the
order its merges imply; the moment-based resolve's opacity is exact, equal
colours come out exact, and with at most three distinct depths the
four-moment bound is the exact fraction of absorbance in front (up to the
moment bias).
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.test_oracle_pins import flat_style

FAR = synth.Hotspot((50.0, 50.0, 50.0), 0.1)


def column(cells_front_to_back_order, importance, W=32):
    """A column of len(importance) unit cells along -z (cell k spans
    z in [-0.1 (n - k), -0.1 (n - k - 1)], so the last cell is the front one),
    listed to the oracle in the given cell order (which fixes the primitive
    order of the faces), with per-cell scalar `importance`."""
    n = len(importance)
    m = synth.box_grid(1, 1, n, size=(1.0, 1.0, 0.1 * n), origin=(-0.5, -0.5, -0.1 * n))
    order = np.asarray(cells_front_to_back_order)
    cam = synth.make_camera((0.0, 0.0, 2.0), (0.0, 0.0, -1.0), W, W, fovy_deg=20.0)
    sc = np.asarray(importance, np.float32)
    return m.xyz, m.hex[order].copy(), sc[order].copy(), cam


def layers(orc, om, st, n):
    """Premultiplied colour and opacity of the cap face at z = -0.1 i
    (i = 0 front .. n back): faces of the column seen from the front."""
    ex = om.export()
    zq = ex["pos_q"][:, 2] / 65536.0
    lo, hi = np.array(st.tf_rgb_lo), np.array(st.tf_rgb_hi)
    out = []
    for i in range(n + 1):
        f = [f for f in range(om.F) if np.all(np.abs(zq[ex["face_v"][f]] + 0.1 * i) < 1e-4)]
        assert len(f) == 1
        t = float(np.mean(ex["t_v"][ex["face_v"][f[0]]]))
        a = st.tf_a_lo + (st.tf_a_hi - st.tf_a_lo) * t
        out.append((a * (lo + (hi - lo) * t), a, f[0]))
    return out


def blend(seq):
    C, T = np.zeros(3), 1.0
    for c, a in seq:
        C += T * c
        T *= 1 - a
    return C, 1 - T


def setup(orc, order, imp, W=32):
    xyz, hexes, sc, cam = column(order, imp, W)
    om = orc.Mesh(xyz, hexes, cell_scalar=sc)
    p = (W // 2) * W + W // 2
    fr = orc.Frame(om, cam.view_proj, W, W, np.array([p]))
    w0, w1 = orc.view_depth_range(om.export()["pos_q"], cam.view_proj)
    return om, fr, cam, w0, w1


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


ST = flat_style(tf_a_lo=0.15, tf_a_hi=0.7, tf_rgb_lo=(0.1, 0.3, 0.9), tf_rgb_hi=(0.95, 0.2, 0.05))


def test_mlab_with_enough_layers_is_exact(orc):
    om, fr, cam, w0, w1 = setup(orc, [0, 1, 2, 3], [0.0, 3.0, 1.0, 2.0])
    exact = fr.shade(FAR, ST)[0]
    for k in (5, 6, 8):
        got = fr.approx(FAR, ST, "mlab", k, w0, w1)
        assert np.abs(got - exact).max() < 1e-12


def test_mlab_non_monotone_arrival_closed_form(orc):
    """Cells listed front, back, middle: the faces arrive (by triangle id) at
    depths 1, 0, 3, 2 (0 = front cap).  With k = 1 or 2 the merges blend the
    layers in the order 0, 1, 3, 2; with k = 3 the result is exact."""
    om, fr, cam, w0, w1 = setup(orc, [2, 0, 1], [1.0, 2.0, 0.0])  # cell 2 is the front cell
    L = layers(orc, om, ST, 3)
    # primitive order of the four cap faces: depth indices by ascending face id
    arrival = [i for _, i in sorted((L[i][2], i) for i in range(4))]
    assert arrival == [1, 0, 3, 2]
    cm, am = blend([(L[i][0], L[i][1]) for i in (0, 1, 3, 2)])
    ce, ae = blend([(L[i][0], L[i][1]) for i in (0, 1, 2, 3)])
    assert np.abs(cm - ce).max() > 1e-3  # the configuration tells the orders apart
    for k in (1, 2):
        got = fr.approx(FAR, ST, "mlab", k, w0, w1)[0]
        assert got[:3] == pytest.approx(cm, abs=1e-12)
        assert got[3] == pytest.approx(am, abs=1e-12)
    got = fr.approx(FAR, ST, "mlab", 3, w0, w1)[0]
    assert got[:3] == pytest.approx(ce, abs=1e-12)


def test_mlab_and_mboit_opacity_is_exact(orc):
    mesh, cams, hots, styles = synth.config0()
    cam = synth.orbit_camera((0.5, 0.5, 0.5), 2.5, 30.0, 20.0, 96, 96)
    hot, st = hots[0], synth.default_style(cam)
    om = orc.Mesh.from_synth(mesh)
    fr = orc.Frame.from_camera(om, cam)
    exact = fr.shade(hot, st)[0]
    w0, w1 = orc.view_depth_range(om.export()["pos_q"], cam.view_proj)
    for method, k in (("mlab", 1), ("mlab", 4), ("mboit", 0)):
        got = fr.approx(hot, st, method, k, w0, w1)
        assert np.abs(got[:, 3] - exact[:, 3]).max() < 1e-6, method  # (opacity clamp 1 - 1e-6)


def test_mboit_equal_colours_are_exact(orc):
    st = flat_style(tf_a_lo=0.25, tf_a_hi=0.25)  # every layer: alpha 0.25, colour tf_rgb_lo
    om, fr, cam, w0, w1 = setup(orc, [0, 1, 2, 3, 4], [0.0, 0.0, 0.0, 0.0, 0.0])
    exact = fr.shade(FAR, st)[0]
    got = fr.approx(FAR, st, "mboit", 0, w0, w1)
    assert np.abs(got - exact).max() < 1e-12


@pytest.mark.parametrize("n", [1, 2])
def test_mboit_few_depths_closed_form(orc, n):
    """With n + 1 <= 3 distinct depths the four moments fix the absorbance
    distribution, so the bound is exact: fragment i sees the absorbance of
    the layers in front plus eta times its own."""
    from oracle import MBOIT_ETA
    imp = [2.0, 0.5, 1.0][:n]
    om, fr, cam, w0, w1 = setup(orc, list(range(n)), imp)
    L = layers(orc, om, ST, n)
    ab = [-np.log1p(-a) for _, a, _ in L]
    C, W = np.zeros(3), 0.0
    for i, (c, a, _) in enumerate(L):
        T = np.exp(-(sum(ab[:i]) + MBOIT_ETA * ab[i]))
        C += T * c
        W += T * a
    A = 1 - np.exp(-sum(ab))
    got = fr.approx(FAR, ST, "mboit", 0, w0, w1)[0]
    assert got[3] == pytest.approx(A, abs=1e-12)
    assert got[:3] == pytest.approx(C * A / W, abs=2e-3)  # (bias towards the reference moments)
    # and with a vanishing bias the bound converges to the exact fraction
    got0 = fr.approx(FAR, ST, "mboit", 0, w0, w1, beta=1e-9)[0]
    assert got0[:3] == pytest.approx(C * A / W, abs=1e-5)
