"""GPU parity of the HIP render path against the FP64 CPU oracle.

All calls go through the C ABI (libhexfc.so via the ctypes binding).
Bar: per-pixel fragment counts and depth-sorted record lists bit-exact;
RGBA within 1e-4 per channel of the oracle's result (or of one of its
alternative results where a fragment sits on a discontinuity within FP32
error, see oracle/hexfc_oracle.c).
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests._parity import RGBA_TOL, gpu_lists, gpu_renderer, log, rgba_mismatch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


def full_compare(orc, mesh, cam, hot, style, tuning=None, ws=1 << 28, label=""):
    log(f"[parity] {label} {mesh.name} {cam.width}x{cam.height} tuning={tuning}")
    ref = orc.render(mesh, cam, hot, style)
    r = gpu_renderer(mesh, ws, tuning)
    c, o, rec = gpu_lists(r, cam)
    assert np.array_equal(c, ref["count"]), f"counts differ at {np.nonzero(c != ref['count'])[0][:10]}"
    assert np.array_equal(o, ref["off"])
    assert np.array_equal(rec, ref["rec"]), "sorted records differ"
    img = r.render(cam, hot, style).cpu().numpy().reshape(-1, 4)
    bad, excl = rgba_mismatch(img, ref["rgba"], ref["ncand"], ref["cand_off"], ref["cand"])
    assert bad.size == 0, (bad[:10], img[bad[:3]], ref["rgba"][bad[:3]])
    assert excl.size <= max(1, 1e-3 * len(c))
    return r, ref, img


def test_config0_full_frame(orc):
    mesh, cams, hots, styles = synth.config0()
    r, ref, img = full_compare(orc, mesh, cams[0], hots[0], styles[0], label="config0")
    assert ref["frame"].nfrag == r.total_fragments()
    # the image is not trivial: focus and context both present
    assert (ref["count"] > 0).mean() > 0.3 and img[:, 3].max() > 0.9


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (16, 16), (32, 8)])
def test_config0_tilings(orc, tile):
    mesh, cams, hots, styles = synth.config0()
    full_compare(orc, mesh, cams[0], hots[0], styles[0], tuning=(tile[0], tile[1], 16), label="tile")


@pytest.mark.parametrize("t_sort", [0, 8, 32, 64])
def test_config0_sort_switch(orc, t_sort):
    mesh, cams, hots, styles = synth.config0()
    full_compare(orc, mesh, cams[0], hots[0], styles[0], tuning=(8, 8, t_sort), label="t_sort")


def test_tilings_bit_identical_rgba():
    mesh, cams, hots, styles = synth.config0()
    imgs = []
    for tile in [(8, 8), (16, 8), (16, 16), (32, 8)]:
        r = gpu_renderer(mesh, 1 << 26, (tile[0], tile[1], 16))
        imgs.append(r.render(cams[0], hots[0], styles[0]).cpu().numpy())
    for im in imgs[1:]:
        assert np.array_equal(im, imgs[0])


def test_determinism_and_multipass():
    """Same frame twice: bitwise equal.  A workspace a fraction of the frame's
    fragments forces several screen passes: bitwise equal to one pass."""
    mesh, cams, hots, styles = synth.scaled_config(16, 320, 200, "jitter", nviews=2)
    r = gpu_renderer(mesh, 1 << 28)
    a = r.render(cams[1], hots[1], styles[1]).cpu().numpy()
    b = r.render(cams[1], hots[1], styles[1]).cpu().numpy()
    assert np.array_equal(a, b)
    F = r.total_fragments()
    small = gpu_renderer(mesh, (F * 8) // 5 + 4096)
    c = small.render(cams[1], hots[1], styles[1]).cpu().numpy()
    st = small.frame_stats()
    log(f"[parity] multipass F={F} passes={st['passes']}")
    assert st["passes"] >= 5
    assert np.array_equal(a, c)


def test_build_needs_whole_frame_in_workspace():
    import paper_2009_06574_amd as hx
    mesh, cams, hots, styles = synth.config0()
    r = gpu_renderer(mesh, 4096)
    with pytest.raises(hx.HexfcError) as e:
        r.build(cams[0])
    assert e.value.status == -4
    # rendering splits the screen instead
    r2 = gpu_renderer(mesh, 1 << 26)
    ref = r2.render(cams[0], hots[0], styles[0]).cpu().numpy()
    r3 = gpu_renderer(mesh, 8 * 40000)
    out = r3.render(cams[0], hots[0], styles[0]).cpu().numpy()
    assert r3.frame_stats()["passes"] > 1
    assert np.array_equal(ref, out)


def test_one_tile_over_budget_is_an_error():
    import paper_2009_06574_amd as hx
    mesh, cams, hots, styles = synth.config0()
    r = gpu_renderer(mesh, 256)
    with pytest.raises(hx.HexfcError) as e:
        r.render(cams[0], hots[0], styles[0])
    assert e.value.status == -4


def test_error_paths():
    import paper_2009_06574_amd as hx
    mesh, cams, hots, styles = synth.config0()
    r = hx.Renderer(0)
    r.set_workspace(1 << 20)
    with pytest.raises(hx.HexfcError) as e:
        r.render(cams[0], hots[0], styles[0])
    assert e.value.status == -6  # no mesh
    with pytest.raises(hx.HexfcError) as e:
        r.resolve(hots[0], styles[0])
    assert e.value.status == -6  # no lists
    r.upload(mesh)
    bad = synth.Camera(view_proj=cams[0].view_proj * 10, width=64, height=64)
    with pytest.raises(hx.HexfcError) as e:
        r.render(bad, hots[0], styles[0])
    assert e.value.status == -2
    with pytest.raises(hx.HexfcError) as e:
        r.render(synth.Camera(view_proj=cams[0].view_proj, width=0, height=64), hots[0], styles[0])
    assert e.value.status == -2
    with pytest.raises(hx.HexfcError) as e:
        r.render(cams[0], synth.Hotspot((0.5, 0.5, 0.5), 0.0), styles[0])
    assert e.value.status == -1
    lv = mesh.cell_edge_level.copy()
    lv[0, 1] = 9
    with pytest.raises(hx.HexfcError) as e:
        r.upload_mesh(mesh.xyz, mesh.hex, None, lv)
    assert e.value.status == -1
    # the failed upload left the previous mesh usable
    r.set_workspace(1 << 26)
    r.render(cams[0], hots[0], styles[0])


def test_watertight_planar_gpu(orc):
    from tests.test_oracle_pins import ortho_planar_setup
    W = 64
    xyz, hexes, vp = ortho_planar_setup(W, 1)
    mesh = synth.Mesh(xyz=xyz, hex=hexes, cell_edge_level=np.zeros((hexes.shape[0], 12), np.uint8))
    cam = synth.Camera(view_proj=vp, width=W, height=W)
    r = gpu_renderer(mesh, 1 << 24)
    c, o, rec = gpu_lists(r, cam)
    assert np.all(c == 2)


@pytest.mark.parametrize("n,a", [(4, 0.3), (20, 0.05)])
def test_equal_alpha_layers_gpu(n, a):
    from tests.test_oracle_pins import column_setup, flat_style
    m, cam = column_setup(n)
    st = flat_style(tf_a_lo=a, tf_a_hi=a)
    r = gpu_renderer(m, 1 << 24)
    img = r.render(cam, synth.Hotspot((50.0, 50.0, 50.0), 0.1), st).cpu().numpy()
    W = cam.width
    px = img[W // 2, W // 2]
    alpha = 1 - (1 - a) ** (n + 1)
    assert abs(px[3] - alpha) < 1e-5
    assert np.abs(px[:3] - np.array(st.tf_rgb_lo) * alpha).max() < 1e-5


def test_ragged_small_viewport(orc):
    mesh, cams, hots, styles = synth.config0()
    cam = synth.orbit_camera((0.5, 0.5, 0.5), 2.5, 50.0, 10.0, 37, 23)
    full_compare(orc, mesh, cam, hots[0], synth.default_style(cam), label="ragged")


def test_maximum_viewport_width(orc):
    """The largest viewport side the ABI accepts (8192) with a ragged 40-pixel
    height, whole frame."""
    mesh, cams, hots, styles = synth.config0()
    cam = synth.orbit_camera((0.5, 0.5, 0.5), 1.2, 30.0, 20.0, 8192, 40, fovy_deg=60.0)
    r, ref, img = full_compare(orc, mesh, cam, hots[0], synth.default_style(cam), label="max width")
    assert (ref["count"] > 0).sum() > 500


@pytest.mark.parametrize("size,fovy", [((1000, 8192), 100.0), ((8192, 8192), 45.0)])
def test_maximum_viewport_sampled(orc, size, fovy):
    """8192 pixels high (a tall frame needs a wide vertical field of view to
    keep the camera matrix within the integer contract), and 8192 x 8192
    (67 M pixels, a million tiles): sampled pixels."""
    mesh, cams, hots, styles = synth.config0()
    cam = synth.orbit_camera((0.5, 0.5, 0.5), 2.5, 30.0, 20.0, size[0], size[1], fovy_deg=fovy)
    r, c = sampled_compare(orc, mesh, cam, hots[0], synth.default_style(cam), ws=1 << 31, nsample=2000)
    assert (c > 0).mean() > 0.05


def test_empty_and_culled(orc):
    mesh, cams, hots, styles = synth.config0()
    st = styles[0]
    st2 = synth.default_style(cams[0], bg=(0.2, 0.3, 0.4))
    # camera looking away from the mesh: every pixel is background
    away = synth.make_camera((0.5, 0.5, 3.0), (0.5, 0.5, 6.0), 64, 48)
    r = gpu_renderer(mesh, 1 << 24)
    img = r.render(away, hots[0], st2).cpu().numpy()
    assert r.total_fragments() == 0
    assert np.all(img == np.array([0.2, 0.3, 0.4, 0.0], np.float32))
    # a mesh with no cells
    empty = synth.Mesh(xyz=mesh.xyz, hex=np.zeros((0, 8), np.int32), cell_edge_level=np.zeros((0, 12), np.uint8))
    r2 = gpu_renderer(empty, 1 << 24)
    img = r2.render(cams[0], hots[0], st2).cpu().numpy()
    assert r2.total_fragments() == 0 and np.all(img[..., 3] == 0)


def test_scaled_config1_multi_view(orc):
    """32^3 jittered grid at 480x270 (several tiles, ragged last tile row)."""
    mesh, cams, hots, styles = synth.scaled_config(32, 480, 270, "jitter", nviews=4)
    for k in (0, 3):
        full_compare(orc, mesh, cams[k], hots[k], styles[k], label=f"c1s view{k}")


def test_scaled_config2_bent(orc):
    mesh, cams, hots, styles = synth.scaled_config(32, 400, 300, "bent", nviews=4)
    full_compare(orc, mesh, cams[1], hots[1], styles[1], label="c2s")


def sampled_compare(orc, mesh, cam, hot, style, ws, nsample=3000, seed=0, tuning=None):
    """Full-size frame on the GPU; the oracle computes a random pixel sample
    plus one full row, one by one."""
    rng = np.random.default_rng(seed)
    W, H = cam.width, cam.height
    pix = np.unique(np.concatenate([rng.integers(0, W * H, nsample), (H // 2) * W + np.arange(W)])).astype(np.int32)
    log(f"[parity] sampled {mesh.name} {W}x{H} samples={pix.size}")
    om = orc.Mesh.from_synth(mesh)
    fr = orc.Frame.from_camera(om, cam, pixels=pix)
    cnt, off, rec = fr.lists()
    rgba, ncand, cand_off, cand = fr.shade(hot, style)
    r = gpu_renderer(mesh, ws, tuning)
    c, o, grec = gpu_lists(r, cam)
    assert np.array_equal(c[pix], cnt)
    for s, p in enumerate(pix):
        assert np.array_equal(grec[o[p]:o[p + 1]], rec[off[s]:off[s + 1]]), p
    assert int(c.astype(np.int64).sum()) == r.total_fragments()
    img = r.render(cam, hot, style).cpu().numpy().reshape(-1, 4)
    bad, excl = rgba_mismatch(img[pix], rgba, ncand, cand_off, cand)
    assert bad.size == 0, (pix[bad[:10]], img[pix[bad[:3]]], rgba[bad[:3]])
    assert excl.size <= max(2, 2e-3 * pix.size)
    return r, c


def test_config1_full_size_sampled(orc):
    mesh, cams, hots, styles = synth.config1()
    r, c = sampled_compare(orc, mesh, cams[2], hots[2], styles[2], ws=4 << 30)
    log(f"[parity] config1 view2 fragments={r.total_fragments()} max list={c.max()}")


def test_config2_full_size_sampled(orc):
    mesh, cams, hots, styles = synth.config2()
    r, c = sampled_compare(orc, mesh, cams[0], hots[0], styles[0], ws=8 << 30)
    log(f"[parity] config2 view0 fragments={r.total_fragments()} max list={c.max()} stats={r.frame_stats()}")


# ---------------------------------------------------------------- shading variants
@pytest.mark.parametrize("variant", ["screen_lens", "depth_cue", "screen_lens_depth_cue_white"])
def test_config0_shading_variants(orc, variant):
    """The screen-space circular lens, the depth cue in the focus region and
    the white background (Section 4, Section 7.1, Section 4.1) against the
    oracle, whole frame."""
    mesh, cams, hots, styles = synth.config0()
    cam = cams[0]
    st = synth.default_style(cam)
    hot = hots[0]
    if "screen_lens" in variant:
        st.lens_mode = 1
        hot = synth.Hotspot((140.0, 110.0, 0.0), 60.0)
    if "depth_cue" in variant:
        st.desaturate = 0.8
    if "white" in variant:
        st.bg = (1.0, 1.0, 1.0)
    full_compare(orc, mesh, cam, hot, st, label=variant)


def test_shading_variant_errors():
    import paper_2009_06574_amd as hx
    mesh, cams, hots, styles = synth.config0()
    r = gpu_renderer(mesh)
    st = synth.default_style(cams[0], lens_mode=2)
    with pytest.raises(hx.HexfcError):
        r.render(cams[0], hots[0], st)
    st = synth.default_style(cams[0], desaturate=1.5)
    with pytest.raises(hx.HexfcError):
        r.render(cams[0], hots[0], st)
    # the learned tail is defined for the object-space lens only
    r.build(cams[0])
    with pytest.raises(hx.HexfcError):
        r.resolve_learned(hots[0], synth.default_style(cams[0], lens_mode=1), np.zeros(5143, np.float32))


# ---------------------------------------------------------------- silhouettes
@pytest.mark.parametrize("sil", [(0.7, 0.02), (1.0, 0.0), (0.35, 0.3)])
def test_config0_silhouettes(orc, sil):
    """White exterior and interior silhouettes of the boundary surface
    (Section 4.2) against the oracle, whole frame: which pixels are
    silhouettes is an integer decision and must agree exactly, the overlay
    to the RGBA bar."""
    mesh, cams, hots, styles = synth.config0()
    st = synth.default_style(cams[0], sil_alpha=sil[0], sil_tau=sil[1], bg=(1.0, 1.0, 1.0))
    r, ref, img = full_compare(orc, mesh, cams[0], hots[0], st, label=f"silhouettes {sil}")
    base = r.render(cams[0], hots[0], synth.default_style(cams[0], bg=(1.0, 1.0, 1.0))).cpu().numpy().reshape(-1, 4)
    changed = np.any(img != base, axis=1)
    ref0 = orc.render(mesh, cams[0], hots[0], synth.default_style(cams[0], bg=(1.0, 1.0, 1.0)))
    ref_changed = np.any(np.abs(ref["rgba"] - ref0["rgba"]) > 0, axis=1)
    log(f"[parity] silhouettes {sil}: {changed.sum()} pixels (oracle {ref_changed.sum()})")
    assert changed.sum() > 50
    assert np.array_equal(changed, ref_changed)


def test_silhouettes_multipass_and_resolve():
    """Silhouettes over several screen passes, and after build + resolve,
    bitwise equal to the one-pass frame."""
    mesh, cams, hots, styles = synth.scaled_config(16, 320, 200, "jitter", nviews=2)
    st = synth.default_style(cams[1], sil_alpha=0.8)
    r = gpu_renderer(mesh, 1 << 28)
    a = r.render(cams[1], hots[1], st).cpu().numpy()
    r.build(cams[1])
    b = r.resolve(hots[1], st).cpu().numpy()
    assert np.array_equal(a, b)
    F = r.total_fragments()
    small = gpu_renderer(mesh, (F * 8) // 5 + 4096)
    c = small.render(cams[1], hots[1], st).cpu().numpy()
    assert small.frame_stats()["passes"] >= 5
    assert np.array_equal(a, c)
    plain = r.render(cams[1], hots[1], styles[1]).cpu().numpy()
    assert np.any(plain != a)


def test_silhouette_errors():
    import paper_2009_06574_amd as hx
    mesh, cams, hots, styles = synth.config0()
    r = gpu_renderer(mesh)
    for kw in ({"sil_alpha": 1.5}, {"sil_alpha": -0.1}, {"sil_alpha": 0.5, "sil_tau": -1.0}):
        with pytest.raises(hx.HexfcError):
            r.render(cams[0], hots[0], synth.default_style(cams[0], **kw))


# ---------------------------------------------------------------- sheet-based LoD on a non-grid mesh
@pytest.mark.parametrize("lod_level", [1, 2])
def test_polygon_prism_with_sheet_lod(orc, lod_level):
    """A twisted pentagon prism (singular centre edges, sheets that cross and
    touch) with its edge levels from the library's sheet-based LoD builder
    (Section 5), rendered whole-frame against the oracle fed the oracle's own
    levels; the two level sets are first checked equal."""
    import paper_2009_06574_amd as hx
    from oracle import lod
    mesh = synth.polygon_prism(5, 6, 8, twist=0.6, amp=0.05, seed=3)
    got, info = hx.build_lod(mesh.hex, mesh.V)
    want, winfo = lod.sheet_lod(mesh.hex)
    assert np.array_equal(got, want) and info["levels"] == winfo["levels"] >= 2
    mesh.cell_edge_level = want
    cam = synth.orbit_camera((0.5, 0.5, 0.5), 2.0, 35.0, 25.0, 256, 224)
    st = synth.default_style(cam, lod=lod_level)
    hot = synth.Hotspot((0.55, 0.5, 0.6), 0.3)
    full_compare(orc, mesh, cam, hot, st, label=f"prism lod={lod_level}")
