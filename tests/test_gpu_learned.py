"""GPU parity of the learned-tail path against the FP64 oracle.

Tail features, head and exact tail composites of the HIP path against
orc_frame_tail; the BF16 MFMA network kernels (forward, loss, backward, Adam)
against oracle/mlp.py, both its exact FP64 definition and its model of the
kernels' BF16 rounding; and the learned resolve's composition and exact
fallback against the exact resolve.  All calls go through the C ABI.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import mlp
from tests._parity import gpu_renderer, log
from tests.test_oracle_mlp import rand_params

pytestmark = pytest.mark.gpu

FEAT_TOL = 1e-5   # abs + rel, FP32 sums of at most a few hundred terms
COMP_TOL = 1e-4   # head / tail composites, as the RGBA bar


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


def hx():
    import paper_2009_06574_amd as m
    return m


def cuda(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def compare_tail_rows(orc, mesh, cam, hot, style, r, K, sample=None):
    out = r.learned_features(hot, style, K, with_target=True)
    pix = out["pix"].cpu().numpy().astype(np.int64)
    head = out["head"].cpu().numpy().astype(np.float64)
    feat = out["feat"].cpu().numpy().astype(np.float64)
    target = out["target"].cpu().numpy().astype(np.float64)
    assert len(np.unique(pix)) == len(pix)
    rows = np.arange(len(pix))
    if sample is not None and len(rows) > sample:
        rows = np.sort(np.random.default_rng(0).choice(rows, sample, replace=False))
    om = orc.Mesh.from_synth(mesh)
    fr = orc.Frame.from_camera(om, cam, pix[rows])
    w0, w1 = orc.view_depth_range(om.export()["pos_q"], cam.view_proj)
    oh, of, ot, has = fr.tail(hot, style, K, w0, w1)
    count = fr.lists()[0]
    _, ncand, _, _ = fr.shade(hot, style)
    log(f"[learned] {mesh.name} rows={len(pix)} compared={len(rows)} K={K} long={int(has.sum())}")
    # lists of at most K fragments: the head is the whole list, no tail features
    short = ~has
    assert np.all(feat[rows[short]] == 0)
    L = has
    g, o = feat[rows[L]], of[L]
    assert np.array_equal(np.rint(np.expm1(g[:, 0])), count[L].astype(np.float64) - K)
    assert np.all(np.abs(g - o) <= FEAT_TOL * (1 + np.abs(o))), np.abs(g - o).max(axis=0)
    # composites: exact wherever no fragment of the pixel is ambiguous
    clean = L & (ncand == 0)
    assert clean.mean() > 0.9 * L.mean()
    dh = np.abs(head[rows[clean]] - oh[clean]).max()
    dt = np.abs(target[rows[clean]] - ot[clean]).max()
    assert dh <= COMP_TOL and dt <= COMP_TOL, (dh, dt)
    return out


def test_tail_features_config0(orc):
    mesh, cams, hots, styles = synth.config0()
    r = gpu_renderer(mesh, tuning=(8, 8, 0))  # every non-empty list is a row
    r.build(cams[0])
    for K in (1, 4, 8):
        compare_tail_rows(orc, mesh, cams[0], hots[0], styles[0], r, K)


def test_tail_features_config1_sampled(orc):
    mesh, cams, hots, styles = synth.config1()
    r = gpu_renderer(mesh, workspace_bytes=1 << 31)
    r.build(cams[3])
    compare_tail_rows(orc, mesh, cams[3], hots[3], styles[3], r, 8, sample=3000)


# ---------------------------------------------------------------- network kernels
def net_inputs(seed, n):
    rng = np.random.default_rng(seed)
    p = rand_params(seed).astype(np.float32).astype(np.float64)
    X = (rng.normal(0, 1, (n, 9)) / p[9:18] + p[:9]).astype(np.float32).astype(np.float64)
    return p, X


@pytest.mark.parametrize("n", [1, 16, 597, 4099])
def test_mlp_forward(n):
    import torch
    p, X = net_inputs(n, n)
    y = hx().mlp_forward(cuda(p, torch.float32), cuda(X, torch.float32)).cpu().numpy().astype(np.float64)
    yb, _ = mlp.forward(p, X, bf16=True)
    y64, _ = mlp.forward(p, X)
    scale = np.abs(y64).max()
    log(f"[mlp] forward n={n} vs bf16 model {np.abs(y - yb).max() / scale:.2e} "
        f"vs fp64 {np.abs(y - y64).max() / scale:.2e}")
    assert np.abs(y - yb).max() <= 2e-3 * scale
    assert np.abs(y - y64).max() <= 2e-2 * scale


def test_mlp_forward_empty():
    import torch
    y = hx().mlp_forward(torch.zeros(mlp.PARAM_COUNT, device="cuda"), torch.zeros((0, 9), device="cuda"))
    assert y.shape == (0, 5)


@pytest.mark.parametrize("conf_tol", [2e-3, 0.05])
def test_mlp_loss(conf_tol):
    import torch
    rng = np.random.default_rng(2)
    n = 1000
    y = rng.normal(0.3, 0.5, (n, 5)).astype(np.float32).astype(np.float64)
    T = rng.uniform(0, 1, (n, 4)).astype(np.float32).astype(np.float64)
    T[:100] = y[:100, :4]  # exact rows: label 1
    T[100:200] = y[100:200, :4] + rng.choice([-1, 1], (100, 4)) * rng.uniform(0, 0.03, (100, 4))
    T = T.astype(np.float32).astype(np.float64)
    err = np.abs(y[:, :4] - T).max(axis=1)
    keep = np.abs(err - conf_tol) > 1e-6  # no label decided by the last bit
    y, T = y[keep], T[keep]
    n = len(y)
    dy, ls = hx().mlp_loss(cuda(y, torch.float32), cuda(T, torch.float32), conf_tol=conf_tol)
    L, dref = mlp.loss_and_dy(y, T, conf_tol)
    assert np.allclose(dy.cpu().numpy(), dref, rtol=1e-5, atol=1e-9)
    assert float(ls.item()) / n == pytest.approx(L, rel=1e-5)


@pytest.mark.parametrize("n", [16, 803, 20000])
def test_mlp_backward(n):
    import torch
    p, X = net_inputs(100 + n, n)
    rng = np.random.default_rng(n)
    y, _ = mlp.forward(p, X)
    T = rng.uniform(0, 1, (n, 4))
    _, dy = mlp.loss_and_dy(y, T)
    dy = dy.astype(np.float32).astype(np.float64)
    g = hx().mlp_backward(cuda(p, torch.float32), cuda(X, torch.float32),
                          cuda(dy, torch.float32)).cpu().numpy().astype(np.float64)
    _, cb = mlp.forward(p, X, bf16=True)
    gb = mlp.backward(p, cb, dy)
    _, c64 = mlp.forward(p, X)
    g64 = mlp.backward(p, c64, dy)
    assert np.all(g[:18] == 0)
    rel_b = np.linalg.norm(g - gb) / np.linalg.norm(gb)
    rel_64 = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    log(f"[mlp] backward n={n} rel vs bf16 model {rel_b:.2e} vs fp64 {rel_64:.2e}")
    assert rel_b <= 2e-3
    assert rel_64 <= 1e-2
    # every parameter block, separately, and element by element against the
    # block's largest gradient (the model reproduces the kernels' BF16 rounding
    # points; the FP32 sums over rows run in another order, which can move an
    # intermediate across a BF16 rounding boundary now and then)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        s = slice(*mlp.OFF[k])
        assert np.linalg.norm(g[s] - g64[s]) <= 2e-2 * np.linalg.norm(g64[s]) + 1e-9, k
        eb = np.abs(g[s] - gb[s]).max() / np.abs(gb[s]).max()
        e64 = np.abs(g[s] - g64[s]).max() / np.abs(g64[s]).max()
        log(f"[mlp] backward n={n} {k}: max element error / block max: vs bf16 model {eb:.2e}, vs fp64 {e64:.2e}")
        assert eb <= 5e-3, (k, eb)
        assert e64 <= 3e-2, (k, e64)


def test_mlp_backward_accumulates():
    import torch
    p, X = net_inputs(5, 64)
    dy = np.random.default_rng(5).normal(0, 1e-2, (64, 5))
    args = (cuda(p, torch.float32), cuda(X, torch.float32), cuda(dy, torch.float32))
    g1 = hx().mlp_backward(*args)
    g2 = hx().mlp_backward(*args, grad=g1.clone())
    # (the order of the FP32 atomic additions across workgroups is not fixed)
    assert float((g2 - 2 * g1).abs().max()) <= 1e-6 * float(g1.abs().max())


def test_adam_step():
    import torch
    rng = np.random.default_rng(9)
    P = mlp.PARAM_COUNT
    p = rng.normal(0, 0.1, P).astype(np.float32)
    m = rng.normal(0, 1e-3, P).astype(np.float32)
    v = rng.uniform(0, 1e-5, P).astype(np.float32)
    g = rng.normal(0, 1e-3, P).astype(np.float32)
    tp, tm, tv = cuda(p), cuda(m), cuda(v)
    hx().mlp_adam_step(tp, tm, tv, cuda(g), step=3, lr=1e-3)
    rp, rm, rv = mlp.adam_step(p.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                               g.astype(np.float64), 3, 1e-3)
    assert np.array_equal(tp.cpu().numpy()[:18], p[:18])
    assert np.allclose(tp.cpu().numpy(), rp, rtol=0, atol=2e-7)
    # FP32 moments: absolute error of a few ulps of their magnitude (beta1 m
    # and (1 - beta1) g may cancel)
    assert np.allclose(tm.cpu().numpy(), rm, rtol=0, atol=1e-6 * np.abs(rm).max())
    assert np.allclose(tv.cpu().numpy(), rv, rtol=0, atol=1e-6 * np.abs(rv).max())


# ---------------------------------------------------------------- learned resolve
def fixed_logit_params(logit, seed=0):
    p = rand_params(seed)
    p[slice(*mlp.OFF["W3"])].reshape(64, 5)[:, 4] = 0.0
    p[mlp.OFF["b3"][0] + 4] = logit
    return p


@pytest.mark.parametrize("t_sort,K", [(8, 8), (16, 8), (0, 4)])
def test_resolve_learned_all_fallback_is_exact(t_sort, K):
    import torch
    mesh, cams, hots, styles = synth.config0()
    r = gpu_renderer(mesh, tuning=(8, 8, t_sort))
    counts = r.build(cams[0], want_counts=True)
    exact = r.resolve(hots[0], styles[0]).clone()
    rows = r.learned_features(hots[0], styles[0], K)
    rgba, mask = r.resolve_learned(hots[0], styles[0], fixed_logit_params(-60.0), K=K, conf_min=0.999)
    torch.cuda.synchronize()
    # pixel confidence = A_head here: only heads of opacity >= 0.999 keep the (invisible) learned tail
    opaque = torch.zeros(counts.numel(), dtype=torch.bool, device=counts.device)
    sel = (1 - (1 - rows["head"][:, 3])) >= 0.999  # the kernel's FP32 expression (sigmoid(-60) = 0 next to 1)
    opaque[rows["pix"].long()[sel & (counts.reshape(-1)[rows["pix"].long()] > K)]] = True
    opaque = opaque.reshape(counts.shape)
    assert torch.equal(mask == 0, opaque)
    assert torch.equal(rgba[~opaque], exact[~opaque])
    d = (rgba[opaque] - exact[opaque]).abs()
    assert d.numel() == 0 or float(d.max()) <= 2e-3
    r.batch_status()
    fb = r.frame_stats()["fallback"]
    long = int(((counts > t_sort)).sum())
    log(f"[learned] fallback t_sort={t_sort} K={K}: {sum(fb)} of {long} long pixels, {int(opaque.sum())} opaque heads")
    assert sum(fb) == long - int(opaque.sum()) and long > 0


@pytest.mark.parametrize("t_sort,K", [(8, 8), (16, 4), (0, 4)])
def test_resolve_learned_composition(t_sort, K):
    import torch
    mesh, cams, hots, styles = synth.config0()
    hot, st = hots[0], styles[0]
    r = gpu_renderer(mesh, tuning=(8, 8, t_sort))
    counts = r.build(cams[0], want_counts=True)
    exact = r.resolve(hot, st).clone()
    p = fixed_logit_params(10.0, seed=3)
    rgba, mask = r.resolve_learned(hot, st, p, K=K, conf_min=0.5)
    rows = r.learned_features(hot, st, K)
    y = hx().mlp_forward(cuda(p, torch.float32), rows["feat"])
    torch.cuda.synchronize()
    H, W = counts.shape
    long = counts > max(t_sort, K)
    assert torch.equal(mask == 0, long)
    # exact where not learned
    assert torch.equal(rgba[~long], exact[~long])
    # learned pixels: head over clamped prediction over the background
    pix = rows["pix"].long()
    cnt = counts.reshape(-1)[pix]
    sel = cnt > K
    h = rows["head"][sel]
    tail = y[sel, :4].clamp(0, 1)
    comp = h + (1 - h[:, 3:4]) * tail
    bg = torch.tensor(list(st.bg) + [0.0], device=comp.device)
    ref = comp + (1 - comp[:, 3:4]) * bg * torch.tensor([1.0, 1.0, 1.0, 0.0], device=comp.device)
    got = rgba.reshape(-1, 4)[pix[sel]]
    assert torch.allclose(got, ref, rtol=0, atol=2e-6)


@pytest.mark.parametrize("layers,kind", [(40, "flat"), (60, "pairs"), (200, "pairs")])
@pytest.mark.parametrize("K", [3, 5, 8])
def test_resolve_learned_head_selection_with_equal_depths(layers, kind, K):
    """The learned resolve finds each pixel's head by selecting the K smallest
    records without sorting; where equal depths straddle the head's end (layers
    coinciding in pairs with K odd, or every layer at one depth) the selection
    must break the tie by triangle id as the sort does.  Its image must equal
    the composition of the full-sort head (learned_features) with the network's
    tail (nearly transparent layers: most heads let the tail through; an opaque
    head adds less than 2^-20 of tail)."""
    import torch
    from tests.test_gpu_long_lists import see_through_style, stack
    m, cam = stack(layers, flat=kind == "flat", pairs=kind == "pairs", seed=K)
    hot = synth.Hotspot((0.0, 0.0, -1.0), 0.6)
    st = see_through_style(cam)
    r = gpu_renderer(m, tuning=(8, 8, 0))
    counts = r.build(cam, want_counts=True)
    p = fixed_logit_params(10.0, seed=K)
    rgba, mask = r.resolve_learned(hot, st, p, K=K, conf_min=0.5)
    rows = r.learned_features(hot, st, K)
    y = hx().mlp_forward(cuda(p, torch.float32), rows["feat"])
    torch.cuda.synchronize()
    pix = rows["pix"].long()
    sel = counts.reshape(-1)[pix] > K
    assert int((rows["head"][sel, 3] < 0.999).sum()) > 0  # heads that let the tail through
    h = rows["head"][sel]
    comp = h + (1 - h[:, 3:4]) * y[sel, :4].clamp(0, 1)
    bg = torch.tensor(list(st.bg) + [0.0], device=comp.device)
    ref = comp + (1 - comp[:, 3:4]) * bg * torch.tensor([1.0, 1.0, 1.0, 0.0], device=comp.device)
    got = rgba.reshape(-1, 4)[pix[sel]]
    d = float((got - ref).abs().max())
    log(f"[learned] head selection {m.name} K={K}: {int(sel.sum())} pixels, max |d| {d:.2e}")
    assert d <= 2e-6


def test_resolve_learned_errors():
    import torch
    mesh, cams, hots, styles = synth.config0()
    r = gpu_renderer(mesh)
    p = fixed_logit_params(0.0)
    with pytest.raises(hx().HexfcError):  # no lists yet
        r.W, r.H = cams[0].width, cams[0].height
        r.resolve_learned(hots[0], styles[0], p)
    r.build(cams[0])
    for kw in (dict(K=0), dict(K=65), dict(conf_min=1.0), dict(conf_min=-0.1)):
        with pytest.raises(hx().HexfcError):
            r.resolve_learned(hots[0], styles[0], p, **kw)
    torch.cuda.synchronize()
