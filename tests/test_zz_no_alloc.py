"""The allocation-free learned resolve against the allocating one.

hexfc_resolve_learned_noalloc runs the kernels of hexfc_resolve_learned with
its per-row staging in a static per-GPU array instead of context-owned
buffers; on the same lists, parameters and thresholds both must give the same
image and mask (to the RGBA bar of the parity tests) and the same fallback
counts.  Two calls in a row share the array, the second on a smaller input,
then a call from another context on the same GPU; a frame with more
long-list pixels than the array holds is refused before anything runs.
All calls go through the C ABI.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import mlp
from tests._parity import gpu_renderer, log
from tests.test_oracle_mlp import rand_params

pytestmark = pytest.mark.gpu

RGBA_TOL = 1e-4
MAX_ROWS = 1 << 20  # HEXFC_NOALLOC_MAX_ROWS


def hx():
    import paper_2009_06574_amd as m
    return m


def head_gated_params(seed=7):
    """Random network whose confidence logit is -60: the pixel confidence is
    the head's opacity, so a threshold splits learned and fallback pixels."""
    p = rand_params(seed)
    p[slice(*mlp.OFF["W3"])].reshape(64, 5)[:, 4] = 0.0
    p[mlp.OFF["b3"][0] + 4] = -60.0
    return p


def long_rows(r):
    return sum(r.frame_stats()["classes"][1:7])


def compare(r, hot, st, p, K, conf_min, what):
    import torch
    got, gmask = r.resolve_learned(hot, st, p, K=K, conf_min=conf_min, noalloc=True)
    torch.cuda.synchronize()
    got, gmask = got.clone(), gmask.clone()
    r.batch_status()
    fb_got = list(r.frame_stats()["fallback"])
    ref, rmask = r.resolve_learned(hot, st, p, K=K, conf_min=conf_min)
    torch.cuda.synchronize()
    r.batch_status()
    fb_ref = list(r.frame_stats()["fallback"])
    rows = long_rows(r)
    d = float((got - ref).abs().max())
    learned = int((rmask == 0).sum())
    log(f"[noalloc] {what}: rows={rows} learned={learned} fallback={sum(fb_ref)} max|d|={d:.3g}")
    assert torch.equal(gmask, rmask)
    assert d <= RGBA_TOL
    assert fb_got == fb_ref
    return rows, learned, sum(fb_ref)


def test_noalloc_matches_allocating_resolve_two_calls():
    mesh, cams, hots, styles = synth.config2()
    p = head_gated_params()
    r = gpu_renderer(mesh, workspace_bytes=1 << 31)
    r.build(cams[5])
    rows1, learned1, fb1 = compare(r, hots[5], styles[5], p, 8, 0.6, "1920x1080 orbit view 5")
    assert 0 < rows1 <= MAX_ROWS and learned1 > 0 and fb1 > 0
    # second call, same context, smaller input: the array keeps the first
    # call's contents beyond the new rows
    small = synth.orbit_views(mesh, 480, 270)[0]
    r.build(small[5])
    rows2, learned2, fb2 = compare(r, hots[5], synth.default_style(small[5]), p, 8, 0.6, "480x270 orbit view 5")
    assert 0 < rows2 < rows1 and learned2 > 0 and fb2 > 0
    # another context on the same GPU shares the array
    mesh0, cams0, hots0, styles0 = synth.config0()
    r0 = gpu_renderer(mesh0, tuning=(8, 8, 4))
    r0.build(cams0[0])
    rows3, _, _ = compare(r0, hots0[0], styles0[0], p, 4, 0.6, "config0, second context")
    assert 0 < rows3 < rows2


def test_noalloc_rejects_more_rows_than_its_scratch():
    import torch
    mesh, cams, hots, styles = synth.config0()
    lo, hi = mesh.bbox()
    c = 0.5 * (lo + hi)
    # eye inside the mesh: every pixel's list is non-empty, and with t_sort = 0
    # every non-empty list is a row of the learned resolve
    cam = synth.make_camera(c, c + np.array([1.0, 0.3, 0.2]), 1920, 1080)
    r = gpu_renderer(mesh, workspace_bytes=1 << 30, tuning=(8, 8, 0))
    r.build(cam)
    rows = long_rows(r)
    assert rows > MAX_ROWS
    p = head_gated_params()
    out = torch.full((1080, 1920, 4), 7.0, device="cuda")
    mask = torch.full((1080, 1920), 9, dtype=torch.uint8, device="cuda")
    with pytest.raises(hx().HexfcError) as e:
        r.resolve_learned(hots[0], styles[0], p, K=4, conf_min=0.5, out=out, mask=mask, noalloc=True)
    assert e.value.status == -4 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all()) and bool((mask == 9).all())  # nothing enqueued
    # the allocating call takes the same frame
    rgba, m = r.resolve_learned(hots[0], styles[0], p, K=4, conf_min=0.5)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(rgba).all())
    log(f"[noalloc] refused {rows} rows (> {MAX_ROWS}), allocating call took them")
