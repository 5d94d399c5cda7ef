"""Batched rendering (one captured HIP graph over many views) and the
autotuner, through the C ABI.  Every view of a batch must equal the same view
rendered alone (bit for bit), on every replay of the graph."""
from __future__ import annotations

import json

import numpy as np
import pytest

import synth
from tests._parity import gpu_renderer, log, rgba_mismatch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


def small_batch(n=8, W=160, H=128, seed=0, N=16):
    mesh = synth.jittered_grid(N, 0.2, 0)
    cams, hots, styles = synth.random_views(mesh, n, W, H, seed)
    return mesh, cams, hots, styles


def singles(r, cams, hots, styles):
    out = []
    frags = 0
    for c, h, s in zip(cams, hots, styles):
        out.append(r.render(c, h, s).cpu().numpy())
        frags += r.total_fragments()
    return np.stack(out), frags


def test_batch_equals_single_views():
    mesh, cams, hots, styles = small_batch()
    r = gpu_renderer(mesh, 1 << 28)
    ref, frags = singles(r, cams, hots, styles)
    img = r.render_batch(cams, hots, styles).cpu().numpy()
    nf, over = r.batch_status()
    log(f"[batch] 8 views fragments={nf}")
    assert not over and nf == frags
    assert np.array_equal(img, ref)


def test_graph_replays_with_eager_work_between():
    """Replay the captured graph with new cameras several times, with eager
    single-view renders and synchronisations in between; every replay must
    equal the eager renders of the same views."""
    import torch
    mesh, cams, hots, styles = small_batch(n=6, seed=1)
    r = gpu_renderer(mesh, 1 << 28)
    out = None
    for rep in range(4):
        cams_r, hots_r, styles_r = synth.random_views(mesh, 6, 160, 128, seed=100 + rep)
        out = r.render_batch(cams_r, hots_r, styles_r, out=out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().copy()
        nf, over = r.batch_status()
        assert not over
        ref, frags = singles(r, cams_r, hots_r, styles_r)  # eager work between replays
        torch.cuda.synchronize()
        assert nf == frags, rep
        assert np.array_equal(got, ref), rep


def test_batch_workspace_overflow_reported():
    import paper_2009_06574_amd as hx
    mesh, cams, hots, styles = small_batch(n=4)
    r = gpu_renderer(mesh, 1 << 28)
    img = r.render_batch(cams, hots, styles)
    nf, _ = r.batch_status()
    small = gpu_renderer(mesh, (nf * 8) // 2)
    with pytest.raises(hx.HexfcError) as e:
        small.render_batch(cams, hots, styles)
    assert e.value.status == -4
    assert img.shape == (4, 128, 160, 4)


def test_batch_tilings_and_sort_switch_bit_identical():
    mesh, cams, hots, styles = small_batch(n=4, seed=3)
    base = None
    for tile in [(8, 8), (16, 8), (16, 16), (32, 8)]:
        r = gpu_renderer(mesh, 1 << 28, (tile[0], tile[1], 16))
        img = r.render_batch(cams, hots, styles).cpu().numpy()
        if base is None:
            base = img
        assert np.array_equal(img, base), tile


def test_autotune_choice_and_cache(tmp_path):
    mesh, cams, hots, styles = small_batch(n=4, seed=5)
    r = gpu_renderer(mesh, 1 << 28)
    ref = r.render_batch(cams, hots, styles).cpu().numpy()
    cache = tmp_path / "tune.json"
    choice = r.autotune(cams, hots, styles, cache_path=cache)
    log(f"[batch] autotune choice {choice}")
    assert (choice[0], choice[1]) in [(8, 8), (16, 8), (16, 16), (32, 8)]
    assert choice[2] in (0, 8, 16, 32, 64)
    data = json.loads(cache.read_text())
    assert len(data) == 1 and list(data.values())[0]["tile_w"] == choice[0]
    # a second tuner reads the cache
    r2 = gpu_renderer(mesh, 1 << 28)
    assert r2.autotune(cams, hots, styles, cache_path=cache) == choice
    img = r2.render_batch(cams, hots, styles).cpu().numpy()
    # the sort switch may change the blend grouping (few ulps), nothing else
    assert np.abs(img - ref).max() < 1e-5
    # single-view tuning lands in the same file under its own key
    r2.autotune(cams[:1], hots[:1], styles[:1], cache_path=cache)
    assert len(json.loads(cache.read_text())) == 2


def test_config3_batch_against_oracle(orc):
    """32 random views of the 64^3 grid at 1024x1024 in one graph; two views
    checked against the oracle on sampled pixels, every view against its
    single-view render on fragment totals."""
    mesh, cams, hots, styles = synth.config3()
    r = gpu_renderer(mesh, 16 << 30)
    img = r.render_batch(cams, hots, styles).cpu().numpy()
    nf, over = r.batch_status()
    log(f"[batch] config3 fragments={nf} overflow={over}")
    assert not over
    om = orc.Mesh.from_synth(mesh)
    rng = np.random.default_rng(0)
    for v in (0, 17):
        pix = rng.choice(1024 * 1024, 1500, replace=False).astype(np.int32)
        fr = orc.Frame.from_camera(om, cams[v], pixels=pix)
        rgba, ncand, cand_off, cand = fr.shade(hots[v], styles[v])
        got = img[v].reshape(-1, 4)[pix]
        bad, excl = rgba_mismatch(got, rgba, ncand, cand_off, cand)
        assert bad.size == 0, (v, pix[bad[:5]])
        assert excl.size <= 3
    # replay with the same views gives the same image
    img2 = r.render_batch(cams, hots, styles).cpu().numpy()
    assert np.array_equal(img, img2)


def test_batch_silhouettes_per_view():
    """Views of one batch with and without silhouettes: each equals its
    single-view render."""
    mesh, cams, hots, styles = small_batch(n=6, seed=2)
    styles = [synth.default_style(c, sil_alpha=(0.6 if k % 2 == 0 else 0.0)) for k, c in enumerate(cams)]
    r = gpu_renderer(mesh, 1 << 28)
    ref, frags = singles(r, cams, hots, styles)
    img = r.render_batch(cams, hots, styles).cpu().numpy()
    nf, over = r.batch_status()
    assert not over and nf == frags
    assert np.array_equal(img, ref)
