"""Pins of the oracle's edge and face colours (Eq. 1, Eq. 2, Eq. 4 with the
focus-edge halo, darkening and accent brightening of Section 4) on a setup
where every quantity is known by construction.

Two unit-square-section cells side by side along x, seen orthographically
along z on a 64 x 64 viewport (so pixel centres map to world points exactly
and the world-space distance from a fragment to each face edge is a known
closed form).  The left cell has importance 0, the right cell 1, so on the
left cell's front face the shared edge (x = 0.5) has importance t_e = 1 and
its three other edges t_e = 0; vertex importance is 0 at x = 0 and 1 at
x = 0.5, so the face importance t_f grows linearly in x (Section 3: maxima
over incident cells).  Single fragments are shaded with the oracle's
one-fragment entry point; nothing here re-derives the oracle's code path:
the expected colours follow from the transfer function, the known t_e / t_f
and the known distances.  A mistake in which edge's importance colours the
line, in the darkening's sign or focus weighting, in the halo band or colour,
or in the brightening fails one of these.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth

W = 64
LO = np.array([0.2, 0.6, 0.9])
HI = np.array([1.0, 0.0, 0.0])
ZF = np.rint(0.1 * 65536) / 65536  # the face plane z = 0.1 after quantisation to 2^-16


@pytest.fixture(scope="module")
def setup(oracle_lib):
    orc = oracle_lib
    m = synth.box_grid(2, 1, 1, size=(1.0, 0.5, 0.1), origin=(0.0, 0.25, 0.0))
    scal = np.array([0.0, 1.0], np.float32)
    om = orc.Mesh(m.xyz, m.hex, cell_scalar=scal, cell_edge_level=m.cell_edge_level)
    # x in [0, 1] -> clip [-1, 1], w = 1: pixel i has its centre at x = (i + 0.5) / W,
    # row j at y = 1 - (j + 0.5) / W
    vp = np.array([[2, 0, 0, -1], [0, 2, 0, -1], [0, 0, 0, 0], [0, 0, 0, 1]], np.float32)
    fr = orc.Frame(om, vp, W, W)
    ex = om.export()
    P = ex["pos_q"].astype(np.float64) / 65536.0
    # the left cell's face in the plane z = 0.1 (the orthographic projection
    # ignores z): corners with x <= 0.5 and z = 0.1
    face = None
    for f, fv in enumerate(ex["face_v"]):
        c = P[fv]
        if np.all(c[:, 2] == ZF) and np.all(c[:, 0] <= 0.5 + 1e-9):
            face = f
    assert face is not None
    # importance of that face's edges, by construction: 1 on x = 0.5, else 0
    fv = ex["face_v"][face]
    for k in range(4):
        a, b = P[fv[k]], P[fv[(k + 1) % 4]]
        on_shared = abs(a[0] - 0.5) < 1e-9 and abs(b[0] - 0.5) < 1e-9
        assert ex["face_te"][face, k] == (1.0 if on_shared else 0.0)
    return dict(orc=orc, fr=fr, face=face, P=P, ex=ex)


def style(**kw):
    st = synth.Style(w_base=0.01, k_focus=0.0, halo_width=0.0, halo_alpha=1.0, darken=0.0, accent_s=1.0,
                     accent_brighten=0.0, delta=2.0, lod=0, tf_rgb_lo=tuple(LO), tf_rgb_hi=tuple(HI),
                     tf_a_lo=0.0, tf_a_hi=0.0, bg=(0.0, 0.0, 0.0))
    for k, v in kw.items():
        setattr(st, k, v)
    return st


def world(i, j):
    return np.array([(i + 0.5) / W, 1.0 - (j + 0.5) / W, ZF])


def frag(s, i, j, hot, st):
    """(rgb, alpha) of the left cell's front-face fragment at pixel (i, j)
    (whichever of its two triangles covers the pixel)."""
    count, off, rec = s["fr"].lists()
    p = j * W + i
    tris = [int(r & 0xffffffff) for r in rec[off[p]:off[p + 1]] if int(r & 0xffffffff) >> 1 == s["face"]]
    assert len(tris) == 1, tris
    out = s["fr"].shade_one(i, j, tris[0], hot, st)
    assert out[4] == 0  # no predicate within rounding of its threshold
    return out[:3], out[3]


def in_focus(i, j):
    return synth.Hotspot(tuple(world(i, j)), 1.0)  # dist = 0: focus 1


FAR = synth.Hotspot((3.0, 3.0, 3.0), 0.1)  # dist >= 1: focus 0


# pixel 31 of the middle row is 1/128 left of the shared edge x = 0.5; pixel 0 is
# 1/128 right of x = 0; both are about 1/4 from the face's horizontal edges
SHARED, LEFT, ROW = (31, 31), (0, 31), 31


@pytest.mark.parametrize("darken", [0.0, 0.25, 0.6])
def test_focus_edge_colour_is_tf_of_its_importance_darkened(setup, darken):
    """Focus 1, an edge within w: opaque, colour TF(t_e) (1 - darken)."""
    st = style(darken=darken)
    rgb, a = frag(setup, *SHARED, in_focus(*SHARED), st)
    assert a == pytest.approx(1.0, abs=1e-12)
    assert rgb == pytest.approx(HI * (1 - darken), abs=1e-12)
    rgb, a = frag(setup, *LEFT, in_focus(*LEFT), st)
    assert a == pytest.approx(1.0, abs=1e-12)
    assert rgb == pytest.approx(LO * (1 - darken), abs=1e-12)


def test_context_edge_colour_is_tf_undarkened(setup):
    """Focus 0: the contextual edge is opaque with colour TF(t_e); the
    darkening applies in focus only."""
    st = style(darken=0.5)
    rgb, a = frag(setup, *SHARED, FAR, st)
    assert a == 1.0 and rgb == pytest.approx(HI, abs=1e-12)
    rgb, a = frag(setup, *LEFT, FAR, st)
    assert a == 1.0 and rgb == pytest.approx(LO, abs=1e-12)


def test_focus_edge_set_uses_importance_threshold(setup):
    """lod above every level: no contextual edges; delta = 0.5 admits only the
    shared edge (t_e = 1) to the focus set.  In focus the shared edge shows,
    the left edge (t_e = 0) does not; in context neither does."""
    st = style(lod=5, delta=0.5)
    rgb, a = frag(setup, *SHARED, in_focus(*SHARED), st)
    assert a == pytest.approx(1.0, abs=1e-12) and rgb == pytest.approx(HI, abs=1e-12)
    rgb, a = frag(setup, *LEFT, in_focus(*LEFT), st)
    assert a == 0.0 and np.all(rgb == 0.0)
    rgb, a = frag(setup, *SHARED, FAR, st)
    assert a == 0.0 and np.all(rgb == 0.0)


@pytest.mark.parametrize("i", [2, 5, 9])
def test_width_gain_in_focus(setup, i):
    """Eq. 1 width law: a fragment at distance d from the left edge draws the
    edge in focus iff d <= (1 + k) w_base, in context iff d <= w_base."""
    d = (i + 0.5) / W
    st = style(w_base=0.05, k_focus=1.0)
    _, a_focus = frag(setup, i, ROW, in_focus(i, ROW), st)
    _, a_ctx = frag(setup, i, ROW, FAR, st)
    assert a_focus == (1.0 if d <= 0.1 else 0.0)
    assert a_ctx == (1.0 if d <= 0.05 else 0.0)


@pytest.mark.parametrize("halo_alpha", [1.0, 0.6])
def test_halo_band_is_white(setup, halo_alpha):
    """Focus 1, transparent faces: in the band w < d <= w + halo_width the
    fragment is white of opacity halo_alpha (premultiplied), beyond it nothing."""
    st = style(w_base=0.01, halo_width=0.02, halo_alpha=halo_alpha, lod=5, delta=-1.0)
    # pixel 1: d = 1.5/64 = 0.0234 (inside the band (0.01, 0.03]); pixel 2: d = 0.039 (outside)
    rgb, a = frag(setup, 1, ROW, in_focus(1, ROW), st)
    assert a == pytest.approx(halo_alpha, abs=1e-12)
    assert rgb == pytest.approx([halo_alpha] * 3, abs=1e-12)
    rgb, a = frag(setup, 2, ROW, in_focus(2, ROW), st)
    assert a == 0.0 and np.all(rgb == 0.0)


def test_halo_scales_with_focus(setup):
    """At focus 1/2 (normalised distance 0.85) the halo band is w < d <=
    w + halo_width / 2 and the halo's opacity is weighted by the focus."""
    st = style(w_base=0.01, halo_width=0.04, halo_alpha=0.8, lod=5, delta=-1.0)
    c = world(1, ROW)
    hot = synth.Hotspot(tuple(c - np.array([0.0, 0.0, 0.85])), 1.0)  # dist = 0.85 -> focus 0.5
    # pixel 1: d = 0.0234 <= 0.01 + 0.02: halo; pixel 2 (d = 0.039) is outside the halved band
    rgb, a = frag(setup, 1, ROW, hot, st)
    assert a == pytest.approx(0.5 * 0.8, abs=1e-9)
    assert rgb == pytest.approx([0.5 * 0.8] * 3, abs=1e-9)
    hot2 = synth.Hotspot(tuple(world(2, ROW) - np.array([0.0, 0.0, 0.85])), 1.0)
    _, a2 = frag(setup, 2, ROW, hot2, st)
    assert a2 == 0.0


@pytest.mark.parametrize("bright", [0.0, 0.2, 0.9])
def test_accent_brightening(setup, bright):
    """Eq. 2 with the accent brightening: no visible edges, far from the
    hotspot (Eq. 3 factor 1).  Within 2/3 w_base of a face edge the face colour
    TF(t_f) is brightened by (1 + b) (clamped to 1) and its opacity multiplied
    by s; t_f = x / 0.5 on this face."""
    s_acc, a_hat = 1.5, 0.4
    st = style(w_base=0.015, lod=5, delta=2.0, accent_s=s_acc, accent_brighten=bright, tf_a_lo=a_hat, tf_a_hi=a_hat)
    x = 0.5 / W  # pixel 0: d = 1/128 <= 0.01
    tf = x / 0.5
    rgb, a = frag(setup, 0, ROW, FAR, st)
    col = np.minimum((LO + (HI - LO) * tf) * (1 + bright), 1.0)
    af = min(1.0, s_acc * a_hat)
    assert a == pytest.approx(af, abs=1e-12)
    assert rgb == pytest.approx(col * af, abs=1e-12)
    # pixel 10 of the middle row (d = 10.5/64 > 0.01 from every edge): no accent
    x = 10.5 / W
    tf = x / 0.5
    rgb, a = frag(setup, 10, ROW, FAR, st)
    assert a == pytest.approx(a_hat, abs=1e-12)
    assert rgb == pytest.approx((LO + (HI - LO) * tf) * a_hat, abs=1e-12)


def test_edge_over_face_eq4(setup):
    """Eq. 4 at focus 1/2: alpha = a_e + (1 - a_e) a_f and colour
    a_e C_e + (1 - a_e) a_f C_f with a_e = focus (focus edge only, lod above
    every level) and the face term far from its own edges unchanged."""
    st = style(w_base=0.02, lod=5, delta=0.5, darken=0.5, tf_a_lo=0.3, tf_a_hi=0.3)
    i = 31
    c = world(i, ROW)
    hot = synth.Hotspot(tuple(c - np.array([0.0, 0.0, 0.85])), 1.0)  # focus 0.5, Eq. 3 factor 0.85^4
    rgb, a = frag(setup, i, ROW, hot, st)
    focus, ae = 0.5, 0.5
    tf = c[0] / 0.5
    af = 0.3 * 0.85 ** 4
    ce = HI * (1 - 0.5 * focus)
    cf = LO + (HI - LO) * tf
    assert a == pytest.approx(ae + (1 - ae) * af, abs=1e-9)
    assert rgb == pytest.approx(ae * ce + (1 - ae) * af * cf, abs=1e-9)
