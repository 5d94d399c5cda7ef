"""Pins of the shading variants the paper describes beside the default
look: the screen-space circular lens (Section 4: a circle with a centre and
radius in screen space, focus 1 at the centre and 0 at its border) and the
depth cue that desaturates far fragments in the focus region (Section 7.1).

A column of equal layers seen head-on gives closed forms: with no edges the
lens only enters through Eq. 3's min(dist, 1)^4; with the lens at half its
radius from a pixel (focus 1, face opacity alpha/16) each layer i at
normalised depth i/n is desaturated by desaturate * i / n.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from tests.test_oracle_pins import column_setup, flat_style


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


def centre_frame(orc, n, W=32, pix=None):
    m, cam = column_setup(n, W)
    om = orc.Mesh.from_synth(m)
    if pix is None:
        pix = np.array([(W // 2) * W + W // 2])
    return orc.Frame.from_camera(om, cam, pix), cam


@pytest.mark.parametrize("d", [0.0, 0.3, 0.8, 1.0, 2.5])
def test_screen_lens_face_opacity(orc, d):
    """Pixel (16, 16) at d lens radii from the lens centre: n + 1 layers of
    opacity a * min(d, 1)^4."""
    n, a, W = 5, 0.4, 32
    fr, cam = centre_frame(orc, n, W)
    st = flat_style(tf_a_lo=a, tf_a_hi=a, lens_mode=1)
    r = 6.0
    hot = synth.Hotspot((16.5 + d * r, 16.5, 0.0), r)
    rgba = fr.shade(hot, st)[0][0]
    ai = a * min(d, 1.0) ** 4
    A = 1 - (1 - ai) ** (n + 1)
    assert rgba[3] == pytest.approx(A, abs=1e-12)
    assert rgba[:3] == pytest.approx(np.array(st.tf_rgb_lo) * A, abs=1e-12)


def test_screen_lens_ignores_depth_and_object_position(orc):
    """The screen-space lens depends on the pixel only: moving the lens's
    (unused) third coordinate changes nothing."""
    fr, cam = centre_frame(orc, 4, pix=np.arange(32 * 32))
    st = synth.default_style(cam, lens_mode=1)
    a = fr.shade(synth.Hotspot((10.0, 20.0, 0.0), 7.0), st)[0]
    b = fr.shade(synth.Hotspot((10.0, 20.0, 5.0), 7.0), st)[0]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("des", [0.0, 0.5, 1.0])
def test_depth_cue_desaturation_closed_form(orc, des):
    n, a, W = 6, 0.3, 32
    fr, cam = centre_frame(orc, n, W)
    c = np.array([0.9, 0.2, 0.1])
    st = flat_style(tf_a_lo=a, tf_a_hi=a, tf_rgb_lo=tuple(c), lens_mode=1, desaturate=des)
    r = 8.0
    hot = synth.Hotspot((16.5 + 0.5 * r, 16.5, 0.0), r)  # dist 0.5: focus 1, face opacity a / 16
    rgba = fr.shade(hot, st)[0][0]
    ai = a * 0.5 ** 4
    lum = 0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2]
    C, T = np.zeros(3), 1.0
    for i in range(n + 1):  # layer i at normalised view depth i / n
        s = des * i / n
        C += T * ai * ((1 - s) * c + s * lum)
        T *= 1 - ai
    assert rgba[3] == pytest.approx(1 - T, abs=1e-12)
    assert rgba[:3] == pytest.approx(C, abs=2e-6)  # (layer depths are quantised to 2^-16)
    if des > 0:
        grey = abs(rgba[0] - rgba[1])
        base = fr.shade(hot, flat_style(tf_a_lo=a, tf_a_hi=a, tf_rgb_lo=tuple(c), lens_mode=1))[0][0]
        assert grey < abs(base[0] - base[1])  # less saturated than without the cue


def test_depth_cue_only_in_focus(orc):
    """Far from the lens (focus 0) the depth cue changes nothing."""
    fr, cam = centre_frame(orc, 4, pix=np.arange(32 * 32))
    hot = synth.Hotspot((0.5, 0.5, 0.0), 3.0)
    st0 = synth.default_style(cam, lens_mode=1)
    st1 = synth.default_style(cam, lens_mode=1, desaturate=1.0)
    a, b = fr.shade(hot, st0)[0], fr.shade(hot, st1)[0]
    far = np.array([((p % 32) - 0.5) ** 2 + ((p // 32) - 0.5) ** 2 > (3.0 + 1.5) ** 2 for p in range(32 * 32)])
    assert np.array_equal(a[far], b[far])
    assert not np.array_equal(a[~far], b[~far]) or np.all(a[~far, 3] == 0)
