"""Pins of the oracle's screen-space silhouettes (Section 4.2, final look):
boundary faces of a grid, the exterior ring of a single cube, and the
interior silhouette where a near cube covers a far one.  The expected sets
come from coverage masks of the cubes rendered separately, not from depth
values."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.test_oracle_pins import flat_style

FAR = synth.Hotspot((50.0, 50.0, 50.0), 0.1)


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_boundary_faces_of_a_grid(orc, N):
    m = synth.box_grid(N, N, N)
    om = orc.Mesh(m.xyz, m.hex)
    b = om.boundary()
    assert b.sum() == 6 * N * N and om.F == 3 * N * N * (N + 1)


def ring(mask):
    """Pixels of mask with a 4-neighbour inside the image that is not in mask."""
    H, W = mask.shape
    out = np.zeros_like(mask)
    for y in range(H):
        for x in range(W):
            if not mask[y, x]:
                continue
            for nx, ny in ((x - 1, y), (x + 1, y), (x, y - 1), (x, y + 1)):
                if 0 <= nx < W and 0 <= ny < H and not mask[ny, nx]:
                    out[y, x] = True
    return out


def cube(lo, size):
    m = synth.box_grid(1, 1, 1, size=(size,) * 3, origin=lo)
    return m.xyz, m.hex


def render(orc, parts, cam, st):
    xyz = np.concatenate([p[0] for p in parts])
    hexes, base = [], 0
    for p in parts:
        hexes.append(p[1] + base)
        base += len(p[0])
    om = orc.Mesh(xyz.astype(np.float32), np.concatenate(hexes).astype(np.int32))
    fr = orc.Frame.from_camera(om, cam)
    rgba = fr.shade(FAR, st)[0].reshape(cam.height, cam.width, 4)
    count = fr.lists()[0].reshape(cam.height, cam.width)
    return rgba, count


CAM = synth.make_camera((0.0, 0.0, 3.0), (0.0, 0.0, 0.0), 48, 48, fovy_deg=40.0)


def test_single_cube_exterior_ring(orc):
    a = 0.6
    st0 = flat_style(tf_a_lo=0.3, tf_a_hi=0.3)
    st1 = flat_style(tf_a_lo=0.3, tf_a_hi=0.3, sil_alpha=a)
    part = [cube((-0.4, -0.35, -0.4), 0.8)]
    base, count = render(orc, part, CAM, st0)
    sil, _ = render(orc, part, CAM, st1)
    expect = ring(count > 0)
    changed = np.any(np.abs(sil - base) > 0, axis=2)
    assert expect.sum() > 20 and np.array_equal(changed, expect)
    e = expect
    assert np.allclose(sil[e, :3], (1 - a) * base[e, :3] + a, atol=1e-15)
    assert np.allclose(sil[e, 3], a + (1 - a) * base[e, 3], atol=1e-15)


def test_interior_silhouette_near_over_far(orc):
    """A near cube in front of a larger far one: the near cube's outline over
    the far cube is an interior silhouette (on the near side only), the far
    cube's outline an exterior one."""
    st0 = flat_style(tf_a_lo=0.3, tf_a_hi=0.3)
    st1 = flat_style(tf_a_lo=0.3, tf_a_hi=0.3, sil_alpha=1.0)
    near = cube((-0.25, -0.2, 0.6), 0.4)
    far = cube((-0.9, -0.85, -1.6), 1.6)
    _, cn = render(orc, [near], CAM, st0)
    _, cf = render(orc, [far], CAM, st0)
    base, _ = render(orc, [near, far], CAM, st0)
    sil, _ = render(orc, [near, far], CAM, st1)
    mn, mf = cn > 0, cf > 0
    assert mn.sum() > 20 and (mn & ~mf).sum() == 0  # the near cube lies inside the far one on screen
    expect = ring(mn | mf) | (mn & ring(mn))  # exterior ring, plus the near outline over the far cube
    changed = np.any(np.abs(sil - base) > 0, axis=2)
    assert np.array_equal(changed, expect)
    # the far cube's pixels next to the near outline are not silhouettes
    assert not np.any(changed & mf & ~mn & ~ring(mn | mf))
