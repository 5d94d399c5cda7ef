"""Single frames without host synchronisation.

After the first frame of a mesh, viewport, tiling and workspace (which waits
once to learn the bin and list sizes and the number of screen passes),
hexfc_render_frame neither waits for the stream nor copies anything to the
host: the passes' tile ranges and every resolve's work come from device
memory.  The proof used here is HIP graph capture (a call that waited or
copied inside a capture would fail it): a captured frame, one pass or a
forced multipass budget, replays bit-identically to the eager frame, several
times, with other eager frames and synchronisations in between.  A frame that
outgrows the learned sizes is flagged and makes the next call grow.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests._parity import gpu_renderer, log

pytestmark = pytest.mark.gpu


def setup(ws_frac=None):
    mesh, cams, hots, styles = synth.scaled_config(16, 320, 200, "jitter", nviews=4)
    big = gpu_renderer(mesh, 1 << 28)
    big.render(cams[1], hots[1], styles[1])
    F = big.total_fragments()
    ws = (1 << 28) if ws_frac is None else int(F * 8 * ws_frac) + 4096
    return mesh, cams, hots, styles, ws


@pytest.mark.parametrize("ws_frac", [None, 0.3])
def test_render_frame_graph_replays(ws_frac):
    import torch
    mesh, cams, hots, styles, ws = setup(ws_frac)
    st = synth.default_style(cams[1], sil_alpha=0.6)
    r = gpu_renderer(mesh, ws)
    ref = r.render(cams[1], hots[1], st).clone()  # first frame: sizes learned (one wait)
    passes = r.frame_stats()["passes"]
    log(f"[frames] eager frame: {passes} passes")
    assert passes == 1 if ws_frac is None else passes >= 4
    for k in (0, 2, 0, 2):  # the other views once flagged, then grown for (no wait)
        r.render(cams[k], hots[0], styles[0])
        r.batch_status()
    out = torch.zeros_like(ref)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.render(cams[1], hots[1], st, out=out)
    torch.cuda.synchronize()
    for rep in range(4):
        out.zero_()
        g.replay()
        other = r.render(cams[rep % 2 * 2], hots[0], styles[0])  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep} differs"
        assert not torch.equal(other, ref)
    fr, over = r.batch_status()
    assert not over


def test_capture_of_an_unsized_frame_is_refused():
    import torch

    import paper_2009_06574_amd as hx
    mesh, cams, hots, styles, ws = setup()
    r = gpu_renderer(mesh, ws)
    out = torch.zeros((cams[1].height, cams[1].width, 4), device="cuda")
    g = torch.cuda.CUDAGraph()
    with pytest.raises(hx.HexfcError) as e:
        with torch.cuda.graph(g):
            r.render(cams[1], hots[1], styles[1], out=out)
    assert e.value.status == -6
    torch.cuda.synchronize()


def test_frame_that_outgrows_its_passes_is_flagged_then_grown():
    """Sized on a view that needs few passes; a closer view needs more: that
    frame is flagged, and the next call (which reads the counters the device
    published, without waiting) launches enough passes."""
    mesh, cams, hots, styles = synth.scaled_config(16, 320, 200, "jitter", nviews=4)
    far = synth.orbit_camera((0.5, 0.5, 0.5), 3.2, 30.0, 20.0, 320, 200)
    near = synth.orbit_camera((0.5, 0.5, 0.5), 1.6, 30.0, 20.0, 320, 200)
    st_far, st_near = synth.default_style(far), synth.default_style(near)
    hot = hots[1]
    probe = gpu_renderer(mesh, 1 << 28)
    probe.render(far, hot, st_far)
    f_far = probe.total_fragments()
    want = probe.render(near, hot, st_near).cpu().numpy()
    f_near = probe.total_fragments()
    log(f"[frames] far {f_far} near {f_near} fragments")
    assert f_near > 2 * f_far
    r = gpu_renderer(mesh, int(f_far * 8 * 0.6) + 4096)  # the far view takes 2 passes
    r.render(far, hot, st_far)
    p_far = r.frame_stats()["passes"]
    r.render(near, hot, st_near)
    _, over = r.batch_status()
    assert over, "the near frame needed more passes than were launched"
    got = r.render(near, hot, st_near).cpu().numpy()
    _, over = r.batch_status()
    st = r.frame_stats()
    log(f"[frames] passes far {p_far}, near {st['passes']}")
    assert not over and st["passes"] > p_far
    assert np.array_equal(got, want)
