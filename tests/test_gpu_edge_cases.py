"""GPU parity on seeded random tiny meshes and the method's degenerate cases.

Each case is a grid of 1 to 27 cells, jittered (strong jitter folds faces
into bow-ties: two fragments of one face at a pixel, ordered by the triangle
bit), with random per-cell importances, edge-level threshold, widths and a
random hotspot, seen by one of five camera kinds:

  0  an ordinary view from outside, random (often ragged) viewport;
  1  grazing: the eye in the plane of a grid layer, so the faces of that layer
     are seen edge-on (zero snapped area, edges through pixel centres);
  2  the eye inside the mesh: vertices behind the near plane (w < 1/16) cull
     the triangles that use them, on both sides;
  3  a 4096-pixel-wide viewport whose frustum cuts the mesh, so vertices land
     outside the guard band (|s| >= 2^17 sub-pixels) and are culled;
  4  strong jitter (folded faces) seen from outside.

Whole frames: counts and sorted records bit-exact, RGBA within 1e-4 of the
oracle's result (or of one of its alternative results where a fragment sits
on a discontinuity within FP32 error).
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests._parity import gpu_lists, log, rgba_mismatch

pytestmark = pytest.mark.gpu

N_CASES = 100


def random_case(seed):
    rng = np.random.default_rng(seed)
    kind = seed % 5
    nx, ny, nz = (int(v) for v in rng.integers(1, 4, 3))
    m = synth.box_grid(nx, ny, nz)
    xyz = m.xyz.astype(np.float64)
    amp = {0: 0.25, 1: 0.0, 2: 0.2, 3: 0.2, 4: 0.9}[kind] / max(nx, ny, nz)
    if amp > 0:
        xyz += rng.uniform(-amp, amp, xyz.shape)
    m.xyz = xyz.astype(np.float32)
    m.cell_scalar = rng.uniform(0, 1, m.C).astype(np.float32) if rng.uniform() < 0.7 else None
    m.name = f"case{seed}k{kind}"
    c = np.array([0.5, 0.5, 0.5])
    if kind == 1:
        # eye in the plane y = j / ny of an unjittered layer, looking across it
        j = int(rng.integers(0, ny + 1))
        y = j / ny
        az = rng.uniform(0, 2 * np.pi)
        eye = np.array([0.5 + 2.2 * np.cos(az), y, 0.5 + 2.2 * np.sin(az)])
        w = int(rng.integers(8, 97))
        cam = synth.make_camera(eye, (0.5, y, 0.5), w, int(np.clip(w * rng.uniform(0.5, 2.0), 8, 96)))
    elif kind == 2:
        eye = c + rng.uniform(-0.3, 0.3, 3)
        d = rng.normal(size=3)
        w = int(rng.integers(16, 97))
        cam = synth.make_camera(eye, eye + d / np.linalg.norm(d), w, int(np.clip(w * rng.uniform(0.5, 2.0), 16, 96)),
                                fovy_deg=float(rng.uniform(40, 100)))
    elif kind == 3:
        # a square 30-degree frustum stretched over 4096 x H pixels: the mesh
        # reaches several frustum widths to the side, beyond +-8192 pixels
        az, el = rng.uniform(0, 2 * np.pi), rng.uniform(-0.5, 0.5)
        eye = c + float(rng.uniform(0.9, 1.4)) * np.array([np.cos(el) * np.sin(az), np.sin(el),
                                                          np.cos(el) * np.cos(az)])
        vp = synth.perspective(30.0, 1.0, 0.1, 10.0) @ synth.look_at(eye, c, (0.0, 1.0, 0.0))
        cam = synth.Camera(view_proj=vp.astype(np.float32), width=4096, height=int(rng.integers(4, 17)),
                           eye=tuple(eye), target=tuple(c), fovy_deg=30.0)
    else:
        w = int(rng.integers(1, 97))
        h = int(np.clip(w * rng.uniform(0.5, 2.0), 1, 96))  # aspect within the matrix limits
        cam = synth.orbit_camera(tuple(c), float(rng.uniform(1.8, 3.0)), float(rng.uniform(0, 360)),
                                 float(rng.uniform(-60, 60)), w, h)
    px = max(cam.pixel_world(), 1e-3)
    st = synth.default_style(cam, w_base=float(rng.uniform(0.3, 3.0)) * px, lod=int(rng.integers(0, 2)),
                             delta=float(rng.uniform(0.2, 1.0)), halo_alpha=float(rng.uniform(0.3, 1.0)),
                             tf_a_lo=float(rng.uniform(0.02, 0.3)), tf_a_hi=float(rng.uniform(0.3, 0.9)))
    st.halo_width = 0.5 * st.w_base
    hot = synth.Hotspot(tuple(c + rng.uniform(-0.5, 0.5, 3)), float(rng.uniform(0.15, 0.8)))
    return m, cam, hot, st


@pytest.fixture(scope="module")
def results(oracle_lib):
    """Runs every case once (one renderer per case) and records what happened."""
    import paper_2009_06574_amd as hx
    out = []
    for seed in range(N_CASES):
        m, cam, hot, st = random_case(seed)
        ref = oracle_lib.render(m, cam, hot, st)
        r = hx.Renderer(0)
        r.set_workspace(1 << 24)
        r.upload(m)
        c, o, rec = gpu_lists(r, cam)
        img = r.render(cam, hot, st).cpu().numpy().reshape(-1, 4)
        out.append(dict(seed=seed, m=m, cam=cam, ref=ref, c=c, o=o, rec=rec, img=img))
        r.close()
    log(f"[edge] {N_CASES} cases, {sum(int(x['c'].sum()) for x in out)} fragments")
    return out


def test_counts_and_order(results):
    for x in results:
        ref = x["ref"]
        assert np.array_equal(x["c"], ref["count"]), (x["m"].name, np.nonzero(x["c"] != ref["count"])[0][:10])
        assert np.array_equal(x["o"], ref["off"]), x["m"].name
        assert np.array_equal(x["rec"], ref["rec"]), x["m"].name


def test_rgba(results):
    excluded = 0
    for x in results:
        ref = x["ref"]
        bad, excl = rgba_mismatch(x["img"], ref["rgba"], ref["ncand"], ref["cand_off"], ref["cand"])
        assert bad.size == 0, (x["m"].name, bad[:10], x["img"][bad[:3]], ref["rgba"][bad[:3]])
        excluded += excl.size
    assert excluded <= 3


def test_cases_reach_the_degenerate_paths(results):
    """The seeds really produce what they are meant to: culled vertices on both
    sides (near plane, guard band), folded faces (two fragments of one face at
    a pixel) and edge-on layers."""
    near = guard = folded = 0
    for x in results:
        fr = x["ref"]["frame"]
        _, _, _, fl = fr.vertices()
        near += int(np.sum(fl == 1))
        guard += int(np.sum(fl == 2))
        rec, off = x["ref"]["rec"], x["ref"]["off"]
        face = (rec & np.uint64(0xffffffff)) >> np.uint64(1)
        for p in np.nonzero(x["c"] > 1)[0]:
            f = face[off[p]:off[p + 1]]
            if np.unique(f).size < f.size:
                folded += 1
    log(f"[edge] vertices behind the near plane {near}, outside the guard band {guard}, "
        f"pixels with two fragments of one face {folded}")
    assert near > 0 and guard > 0 and folded > 0
