"""Pins of the FP64 CPU oracle against facts the paper and mathematics fix.

Every test here runs on the CPU.  None of them re-derives the oracle's own
formulas: they use closed forms, invariants, an independent world-space ray
caster (tests/_raycast.py) and brute force on tiny inputs, chosen so that a
dropped term, a flipped sign, a wrong index or a transposed operand in the
oracle fails at least one of them.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import synth
from tests import _raycast as rc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


def unit_cube():
    return np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                     (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)], dtype=np.float64)


def rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = math.cos(ax), math.sin(ax), math.cos(ay), math.sin(ay), math.cos(az), math.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


# ------------------------------------------------------------------ Section 3: deformation measure

def test_scaled_jacobian_cube_and_cuboid(orc):
    assert orc.scaled_jacobian(unit_cube()) == pytest.approx(1.0, abs=1e-15)
    assert orc.scaled_jacobian(unit_cube() * np.array([0.3, 2.0, 7.5])) == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("s", [0.1, 0.5, 1.0, 3.0])
def test_scaled_jacobian_shear_closed_form(orc, s):
    c = unit_cube()
    c[:, 0] += s * c[:, 1]  # x' = x + s y
    assert orc.scaled_jacobian(c) == pytest.approx(1.0 / math.sqrt(1 + s * s), rel=1e-12)


def test_scaled_jacobian_rigid_and_scale_invariant(orc):
    rng = np.random.default_rng(3)
    c = unit_cube() + rng.uniform(-0.2, 0.2, size=(8, 3))
    ref = orc.scaled_jacobian(c)
    for k in range(5):
        R = rot(*rng.uniform(0, 2 * math.pi, 3))
        c2 = (c @ R.T) * rng.uniform(0.1, 10.0) + rng.normal(size=3)
        assert orc.scaled_jacobian(c2) == pytest.approx(ref, rel=1e-12, abs=1e-13)


def test_scaled_jacobian_inverted_corner_is_negative(orc):
    c = unit_cube()
    c[6] = (0.2, 0.2, 0.2)  # corner 6 pushed through the cell centre
    assert orc.scaled_jacobian(c) < 0


# ------------------------------------------------------------------ mesh attributes

@pytest.mark.parametrize("N", [1, 2, 3, 8])
def test_face_count_closed_form(orc, N):
    m = synth.jittered_grid(N, 0.2, 0) if N > 1 else synth.box_grid(1, 1, 1)
    om = orc.Mesh.from_synth(m)
    assert om.V == (N + 1) ** 3
    assert om.C == N ** 3
    assert om.F == 3 * N * N * (N + 1)


def test_face_dedup_two_cells_golden(orc):
    """Two cells sharing a face: 11 faces in first-seen order (hand-derived)."""
    with open(os.path.join(GOLD, "two_cells.json")) as f:
        g = json.load(f)
    xyz = np.asarray(g["xyz"], np.float32)
    hexes = np.asarray(g["hex"], np.int32)
    om = orc.Mesh(xyz, hexes)
    ex = om.export()
    assert om.F == len(g["faces"])
    assert ex["face_v"].tolist() == g["faces"]


def test_importance_max_propagation(orc):
    """One cell of importance 1, all others 0: exactly that cell's 8 vertices
    and 12 edges carry 1 (Section 3: max over incident cells)."""
    m = synth.box_grid(3, 3, 3)
    sc = np.zeros(m.C, np.float32)
    hot = 13  # the centre cell
    sc[hot] = 5.0
    om = orc.Mesh(m.xyz, m.hex, cell_scalar=sc)
    ex = om.export()
    assert ex["t_cell"][hot] == 1.0 and ex["t_cell"].sum() == 1.0
    hv = set(m.hex[hot].tolist())
    assert set(np.nonzero(ex["t_v"] == 1.0)[0].tolist()) == hv
    assert np.all(ex["t_v"][[v for v in range(m.V) if v not in hv]] == 0.0)
    edges = {tuple(sorted((int(m.hex[hot, a]), int(m.hex[hot, b])))) for a, b in synth.CELL_EDGES}
    fv, fte = ex["face_v"], ex["face_te"]
    for f in range(om.F):
        for k in range(4):
            e = tuple(sorted((int(fv[f, k]), int(fv[f, (k + 1) % 4]))))
            assert fte[f, k] == (1.0 if e in edges else 0.0)


def test_importance_is_one_minus_sj_normalised(orc):
    """Undistorted cells (SJ = 1) get importance 0; the most sheared cell gets 1."""
    m = synth.box_grid(2, 1, 1)
    xyz = m.xyz.astype(np.float64).copy()
    right = xyz[:, 0] > 0.75  # shear only the right cell's far face
    xyz[right & (xyz[:, 1] > 0.5), 0] += 0.25
    om = orc.Mesh(xyz.astype(np.float32), m.hex)
    t = om.export()["t_cell"]
    assert t.tolist() == [0.0, 1.0]


def test_inconsistent_edge_levels_rejected(orc):
    m = synth.box_grid(2, 1, 1)
    lv = np.zeros((2, 12), np.uint8)
    lv[0, 1] = 3  # edge (1,2) of cell 0 is edge (0,3) of cell 1, which says 0
    with pytest.raises(orc.OracleError):
        orc.Mesh(m.xyz, m.hex, cell_edge_level=lv)


def test_out_of_range_rejected(orc):
    m = synth.box_grid(1, 1, 1)
    with pytest.raises(orc.OracleError):
        orc.Mesh(m.xyz * 5.0, m.hex)
    bad = m.hex.copy()
    bad[0, 0] = 99
    with pytest.raises(orc.OracleError):
        orc.Mesh(m.xyz, bad)


# ------------------------------------------------------------------ coverage: fill rule

def ortho_planar_setup(W, seed):
    """A 1-cell-thick quad grid, projected orthographically along z, whose
    vertices sit on the sub-pixel lattice (many edges through pixel centres)."""
    rng = np.random.default_rng(seed)
    n = 12
    m = synth.box_grid(n, n, 1, size=(1.5, 1.5, 0.1), origin=(-0.25, -0.25, 0.0))
    xyz = m.xyz.astype(np.float64)
    top = xyz[:, 2] > 0.05
    # jitter interior columns by whole sub-pixels (1/(16 W) world units)
    col = np.round((xyz[:, 0] + 0.25) / 0.125).astype(int) + 100 * np.round((xyz[:, 1] + 0.25) / 0.125).astype(int)
    interior = (np.abs(xyz[:, 0] + 0.25) > 1e-9) & (np.abs(xyz[:, 0] - 1.25) > 1e-9) & \
               (np.abs(xyz[:, 1] + 0.25) > 1e-9) & (np.abs(xyz[:, 1] - 1.25) > 1e-9)
    jit = {}
    for c in np.unique(col):
        jit[c] = rng.integers(-40, 41, size=2) / (16.0 * W)
    for v in range(xyz.shape[0]):
        if interior[v]:
            xyz[v, :2] += jit[col[v]]
    # shift the lattice by half a pixel so unjittered vertices sit on pixel
    # centres, then snap every coordinate to whole sub-pixels
    xyz[:, :2] += 8.0 / (16 * W)
    xyz[:, :2] = np.round(xyz[:, :2] * 16 * W) / (16 * W)
    vp = np.array([[2, 0, 0, -1], [0, 2, 0, -1], [0, 0, 0, 0], [0, 0, 0, 1]], np.float32)
    return xyz.astype(np.float32), m.hex, vp


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_watertight_planar_tiling(orc, seed):
    """A planar tiling covers every pixel centre exactly once per layer: no
    cracks, no double hits, whatever edges and vertices pass through centres."""
    W = 64
    xyz, hexes, vp = ortho_planar_setup(W, seed)
    om = orc.Mesh(xyz, hexes)
    fr = orc.Frame(om, vp, W, W)
    count, off, rec = fr.lists()
    sx, sy, q, fl = fr.vertices()
    # at least some lattice vertices sit exactly on pixel centres
    assert np.any(((sx - 8) % 16 == 0) & ((sy - 8) % 16 == 0))
    assert np.all(count == 2), np.unique(count, return_counts=True)


def test_fill_rule_single_pixel_square(orc):
    """A square whose corners are 4 neighbouring pixel centres covers exactly
    one of those 4 centres (the half-open rule)."""
    W = 8
    s = 1.0 / (16 * W)
    x0, y0 = (16 * 2 + 8) * s, (16 * 3 + 8) * s
    m = synth.box_grid(1, 1, 1, size=(16 * s, 16 * s, 0.1), origin=(x0, y0, 0.0))
    vp = np.array([[2, 0, 0, -1], [0, 2, 0, -1], [0, 0, 0, 0], [0, 0, 0, 1]], np.float32)
    om = orc.Mesh(m.xyz, m.hex)
    fr = orc.Frame(om, vp, W, W)
    count, _, _ = fr.lists()
    # front and back quads each own exactly one of the four corner centres
    assert count.sum() == 2
    assert np.count_nonzero(count) == 1


# ------------------------------------------------------------------ coverage and order vs world-space ray casting

@pytest.fixture(scope="module")
def cfg0_small(orc):
    mesh, cams, hots, styles = synth.config0()
    cam = synth.orbit_camera((0.5, 0.5, 0.5), 2.5, 30.0, 20.0, 96, 96)
    om = orc.Mesh.from_synth(mesh)
    fr = orc.Frame.from_camera(om, cam)
    ex = om.export()
    P = ex["pos_q"].astype(np.float64) / 65536.0
    fv = ex["face_v"].astype(np.int64)
    tris = []
    for f in fv:
        tris.append((f[0], f[1], f[2]))
        tris.append((f[0], f[2], f[3]))
    hits, near = rc.raycast(P, tris, cam.view_proj, cam.width, cam.height, band=1.0)
    eye, dirs = rc.pixel_rays(cam.view_proj, cam.width, cam.height)
    return dict(mesh=mesh, cam=cam, om=om, fr=fr, hits=hits, near=near, P=P, tris=tris, ex=ex,
                eye=eye, dirs=dirs)


def test_counts_match_world_space_raycast(cfg0_small):
    d = cfg0_small
    count, off, rec = d["fr"].lists()
    far = ~d["near"]
    assert far.mean() > 0.5
    rc_count = np.array([len(h) for h in d["hits"]])
    bad = np.nonzero(far & (rc_count != count))[0]
    assert bad.size == 0, (bad[:10], rc_count[bad[:10]], count[bad[:10]])
    assert count.sum() > 10000


def test_order_matches_world_space_depth(cfg0_small):
    """Sorted lists are front to back: their triangle order equals the order of
    the world-space hit distances (near-equal distances may come in either
    order; they are resolved by triangle id)."""
    d = cfg0_small
    count, off, rec = d["fr"].lists()
    checked = 0
    for p in np.nonzero(~d["near"])[0]:
        h = sorted(d["hits"][p])
        tri_orc = [int(r & 0xffffffff) for r in rec[off[p]:off[p + 1]]]
        if len(h) != len(tri_orc):
            continue
        tt = dict((tid, t) for t, tid in h)
        seq = [tt[t] for t in tri_orc]
        for a, b in zip(seq, seq[1:]):
            assert b >= a - 1e-6 * a, (p, seq)
        checked += 1
    assert checked > 1000


def test_depth_key_monotone_in_distance(cfg0_small):
    """Depth field of the records grows with world distance along the ray."""
    d = cfg0_small
    count, off, rec = d["fr"].lists()
    depth = (rec >> np.uint64(32)).astype(np.int64)
    for p in np.nonzero(~d["near"] & (count > 3))[0][:200]:
        tt = dict((tid, t) for t, tid in d["hits"][p])
        ds = depth[off[p]:off[p + 1]]
        ts = [tt[int(r & 0xffffffff)] for r in rec[off[p]:off[p + 1]]]
        assert np.all(np.diff(ds) >= 0)
        order = np.argsort(ts, kind="stable")
        assert np.all(np.diff(ds[order]) >= -1)


def test_permutation_invariance(orc, cfg0_small):
    """Shuffling the cell order permutes face/triangle ids but leaves every
    pixel's fragment count, depth-key multiset and colour unchanged."""
    d = cfg0_small
    mesh, cam = d["mesh"], d["cam"]
    rng = np.random.default_rng(7)
    perm = rng.permutation(mesh.C)
    om2 = orc.Mesh(mesh.xyz, mesh.hex[perm], None, mesh.cell_edge_level[perm])
    fr2 = orc.Frame.from_camera(om2, cam)
    c1, o1, r1 = d["fr"].lists()
    c2, o2, r2 = fr2.lists()
    assert np.array_equal(c1, c2)
    k1 = r1 >> np.uint64(32)
    k2 = r2 >> np.uint64(32)
    assert np.array_equal(k1, k2)  # lists sorted by key first: key sequences agree
    hot = synth.Hotspot((0.5, 0.5, 0.5), 0.3)
    st = synth.default_style(synth.orbit_camera((0.5, 0.5, 0.5), 2.5, 30.0, 20.0, 256, 256))
    rgba1 = d["fr"].shade(hot, st)[0]
    rgba2 = fr2.shade(hot, st)[0]
    # pixels with equal adjacent keys may blend in another order
    tie = np.zeros(len(c1), bool)
    for p in range(len(c1)):
        kk = k1[o1[p]:o1[p + 1]]
        tie[p] = np.any(kk[1:] == kk[:-1])
    assert np.abs(rgba1 - rgba2)[~tie].max() < 1e-12


def test_repeated_sample_pixels_rejected(orc, cfg0_small):
    d = cfg0_small
    with pytest.raises(orc.OracleError):
        orc.Frame.from_camera(d["om"], d["cam"], pixels=np.array([5, 7, 5], np.int32))


def test_tile_order_independence_of_sample_sets(orc, cfg0_small):
    """Rendering a pixel subset gives the same lists as the full frame."""
    d = cfg0_small
    c1, o1, r1 = d["fr"].lists()
    pix = np.array([0, 5, 4000, 4001, 9215, 4660, 4661, 3333], np.int32)
    fr2 = orc.Frame.from_camera(d["om"], d["cam"], pixels=pix)
    c2, o2, r2 = fr2.lists()
    for s, p in enumerate(pix):
        assert c2[s] == c1[p]
        assert np.array_equal(r2[o2[s]:o2[s + 1]], r1[o1[p]:o1[p + 1]])


# ------------------------------------------------------------------ shading closed forms (Eq. 1-4)

def column_setup(n, W=32, fovy=20.0):
    """n unit cells stacked along the view axis, seen head-on from +z."""
    m = synth.box_grid(1, 1, n, size=(1.0, 1.0, 0.1 * n), origin=(-0.5, -0.5, -0.1 * n))
    cam = synth.make_camera((0.0, 0.0, 2.0), (0.0, 0.0, -1.0), W, W, fovy_deg=fovy)
    return m, cam


def flat_style(**kw):
    st = synth.Style(w_base=1e-4, k_focus=0.0, halo_width=0.0, darken=0.0, accent_s=1.0,
                     accent_brighten=0.0, delta=2.0, lod=100, tf_rgb_lo=(0.2, 0.6, 0.9),
                     tf_rgb_hi=(1.0, 0.0, 0.0), tf_a_lo=0.3, tf_a_hi=0.3, bg=(0.0, 0.0, 0.0))
    for k, v in kw.items():
        setattr(st, k, v)
    return st


@pytest.mark.parametrize("n,a", [(1, 0.3), (4, 0.3), (9, 0.15), (20, 0.05)])
def test_equal_alpha_layers_closed_form(orc, n, a):
    """n+1 faces of equal opacity a: alpha = 1-(1-a)^(n+1), colour = c*alpha."""
    m, cam = column_setup(n)
    st = flat_style(tf_a_lo=a, tf_a_hi=a)
    far = synth.Hotspot((50.0, 50.0, 50.0), 0.1)
    r = orc.render(m, cam, far, st)
    W = cam.width
    centre = [(W // 2) * W + W // 2, (W // 2 - 1) * W + W // 2 - 1]
    for p in centre:
        assert r["count"][p] == n + 1
        alpha = 1 - (1 - a) ** (n + 1)
        assert r["rgba"][p, 3] == pytest.approx(alpha, abs=1e-12)
        assert r["rgba"][p, :3] == pytest.approx(np.array(st.tf_rgb_lo) * alpha, abs=1e-12)


def test_opaque_front_layer_gives_its_colour(orc):
    m, cam = column_setup(5)
    st = flat_style(tf_a_lo=1.0, tf_a_hi=1.0, bg=(0.3, 0.3, 0.3))
    r = orc.render(m, cam, synth.Hotspot((50.0, 50.0, 50.0), 0.1), st)
    p = (cam.width // 2) * cam.width + cam.width // 2
    assert r["rgba"][p].tolist() == pytest.approx(list(st.tf_rgb_lo) + [1.0], abs=1e-15)


def test_background_shows_through_empty_pixels(orc):
    m, cam = column_setup(2, fovy=60.0)
    st = flat_style(bg=(0.1, 0.2, 0.3))
    r = orc.render(m, cam, synth.Hotspot((50.0, 50.0, 50.0), 0.1), st)
    empty = r["count"] == 0
    assert empty.any()
    assert np.all(r["rgba"][empty] == np.array([0.1, 0.2, 0.3, 0.0]))


def test_smoothstep_values(orc):
    assert orc.smoothstep(0.7, 1.0, 0.7) == 0.0
    assert orc.smoothstep(0.7, 1.0, 0.85) == pytest.approx(0.5, abs=1e-15)
    assert orc.smoothstep(0.7, 1.0, 1.0) == 1.0
    assert orc.smoothstep(0.7, 1.0, 0.2) == 0.0
    assert orc.smoothstep(0.7, 1.0, 3.0) == 1.0


def ray_points(d, p):
    """World hit points of pixel p (from the independent ray caster)."""
    return {tid: d["eye"] + t * d["dirs"][p] for t, tid in d["hits"][p]}


def test_face_opacity_vanishes_at_focus_centre(orc, cfg0_small):
    """Eq. 3: alpha_f = alpha_hat * dist^4 -> 0 at the hotspot centre, and
    alpha_hat far away (no edges drawn)."""
    d = cfg0_small
    count, off, rec = d["fr"].lists()
    p = int(np.nonzero(~d["near"] & (count > 4))[0][0])
    pts = ray_points(d, p)
    tri = int(rec[off[p]] & 0xffffffff)
    st = flat_style(tf_a_lo=0.4, tf_a_hi=0.4)
    at_centre = d["fr"].shade_one(p % d["cam"].width, p // d["cam"].width, tri,
                                  synth.Hotspot(tuple(pts[tri]), 0.2), st)
    # the hit point differs from the snapped-vertex interpolation by < 1/16 px
    assert at_centre[3] < 0.4 * (0.002 / 0.2) ** 4
    far = d["fr"].shade_one(p % d["cam"].width, p // d["cam"].width, tri,
                            synth.Hotspot((9.0, 9.0, 9.0), 0.2), st)
    assert far[3] == pytest.approx(0.4, abs=1e-15)
    # half-way: dist = 0.5 -> alpha_hat / 16
    c = pts[tri] + np.array([0.1, 0.0, 0.0])
    half = d["fr"].shade_one(p % d["cam"].width, p // d["cam"].width, tri, synth.Hotspot(tuple(c), 0.2), st)
    assert half[3] == pytest.approx(0.4 / 16, rel=0.05)


def test_edge_alpha_reduces_to_eq1(orc, cfg0_small):
    """With halo and darkening off and transparent faces, every fragment's
    alpha is alpha_e in {0, focus, 1} (Eq. 1), with focus from the independent
    world-space hit point; with focus 0 only contextual edges remain."""
    d = cfg0_small
    count, off, rec = d["fr"].lists()
    W = d["cam"].width
    hot = synth.Hotspot((0.5, 0.5, 0.5), 0.35)
    st = synth.default_style(d["cam"], halo_width=0.0, darken=0.0, tf_a_lo=0.0, tf_a_hi=0.0,
                             accent_s=1.0, w_base=3 * d["cam"].pixel_world())
    seen = {0: 0, 1: 0, "focus": 0}
    for p in np.nonzero(~d["near"] & (count > 0))[0][::7]:
        pts = ray_points(d, p)
        for r in rec[off[p]:off[p + 1]]:
            tri = int(r & 0xffffffff)
            if tri not in pts:
                continue
            out = d["fr"].shade_one(p % W, p // W, tri, hot, st)
            if out[4] != 0:
                continue
            dist = np.linalg.norm(pts[tri] - np.array(hot.center)) / hot.radius
            u = min(max((dist - 0.7) / 0.3, 0.0), 1.0)
            focus = 1 - u * u * (3 - 2 * u)
            a = out[3]
            # focus from the hit point; the snapped interpolation moves it by < 0.02
            ok = [abs(a) < 1e-12, abs(a - 1) < 1e-12, abs(a - focus) < 0.02, abs(a - (1 - focus)) < 0.02]
            assert any(ok), (p, tri, a, focus)
            if ok[0]:
                seen[0] += 1
            elif ok[1]:
                seen[1] += 1
            else:
                seen["focus"] += 1
    assert seen[0] > 0 and seen[1] > 0 and seen["focus"] > 0, seen


def test_no_edges_when_lod_and_delta_exclude_all(orc, cfg0_small):
    """lod above every level and delta > 1: no edge fragments (alpha_e = 0),
    so alpha is the face term alone."""
    d = cfg0_small
    count, off, rec = d["fr"].lists()
    W = d["cam"].width
    st = synth.default_style(d["cam"], lod=99, delta=1.5, accent_s=1.0, tf_a_lo=0.0, tf_a_hi=0.0)
    hot = synth.Hotspot((0.5, 0.5, 0.5), 0.3)
    for p in np.nonzero(count > 0)[0][::37]:
        for r in rec[off[p]:off[p + 1]]:
            assert d["fr"].shade_one(p % W, p // W, int(r & 0xffffffff), hot, st)[3] == 0.0


def test_accentuation_scales_face_opacity(orc, cfg0_small):
    """Eq. 2: near any face edge (d <= 2/3 w_base) alpha_f is multiplied by s
    (no visible edges, focus 0); elsewhere it is unchanged."""
    d = cfg0_small
    count, off, rec = d["fr"].lists()
    W = d["cam"].width
    hot = synth.Hotspot((9.0, 9.0, 9.0), 0.3)
    base = synth.default_style(d["cam"], lod=99, delta=1.5, accent_s=1.0, tf_a_lo=0.2, tf_a_hi=0.2,
                               w_base=4 * d["cam"].pixel_world())
    acc = synth.default_style(d["cam"], lod=99, delta=1.5, accent_s=2.5, tf_a_lo=0.2, tf_a_hi=0.2,
                              w_base=4 * d["cam"].pixel_world())
    ratios = set()
    for p in np.nonzero(count > 0)[0][::11]:
        for r in rec[off[p]:off[p + 1]]:
            tri = int(r & 0xffffffff)
            a0 = d["fr"].shade_one(p % W, p // W, tri, hot, base)
            a1 = d["fr"].shade_one(p % W, p // W, tri, hot, acc)
            if a1[4]:
                continue
            ratios.add(round(a1[3] / a0[3], 9))
    assert ratios == {1.0, 2.5}
