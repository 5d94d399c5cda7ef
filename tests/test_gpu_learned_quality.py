"""Quality of the trained learned-tail network on views it was not trained on.

The shipped network (paper_2009_06574_amd/weights/tail_k8.npz, K = 8) was
trained on random views with seeds 1..1000 of the 2.1 M-cell bent and sheared
grid and of the 64^3 jittered grid at 1920x1080; here it resolves held-out
views (seeds 1001..1004) of the bent grid.  Against the exact resolve of the
same lists (RGB PSNR of the final frame), the learned resolve with pixel
confidence threshold 0.5 must reach 45 dB on every view, and beat both
learning-free tails built from the same head: K-truncation (the tail
dropped) and the proxy tail alone (the network's own ordered proxy-composite
input, features f4..f7) — the comparison an analytic tail gives.  Both
baselines keep the exact result wherever the list has at most K fragments,
so the gains are measured on the long lists only.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests._parity import gpu_renderer, log

pytestmark = pytest.mark.gpu

SEEDS = (1001, 1002, 1003, 1004)
PSNR_MIN = 45.0          # dB, every held-out view
GAIN_TRUNC_MIN = 10.0    # dB over K-truncation, mean over the views
GAIN_PROXY_MIN = 2.0     # dB over the proxy tail, mean over the views


def test_learned_tail_quality_on_held_out_views():
    import torch

    from paper_2009_06574_amd import tail
    p_np, meta = tail.load_weights()
    K = int(meta["K"])
    params = torch.tensor(p_np, device="cuda")
    mesh, _, _, _ = synth.config2()
    r = gpu_renderer(mesh, workspace_bytes=1 << 32)
    rgb = slice(0, 3)
    res = []
    for cam, hot, st in tail._views(mesh, SEEDS, 1920, 1080):
        r.build(cam)
        exact = r.resolve(hot, st).clone()
        base = tail.baselines(r, hot, st, K, exact)
        learned, mask = r.resolve_learned(hot, st, params, K, 0.5)
        torch.cuda.synchronize()
        r.batch_status()
        fb = sum(r.frame_stats()["fallback"])
        q = dict(learned=tail.psnr(learned[..., rgb], exact[..., rgb]),
                 truncated=tail.psnr(base["truncated"][..., rgb], exact[..., rgb]),
                 proxy=tail.psnr(base["proxy"][..., rgb], exact[..., rgb]),
                 learned_px=int((mask == 0).sum()), fallback=fb)
        log(f"[quality] {q}")
        res.append(q)
        assert np.isfinite(q["learned"]) and q["learned"] >= PSNR_MIN, q
        assert q["learned_px"] > 0
    gain_t = np.mean([q["learned"] - q["truncated"] for q in res])
    gain_p = np.mean([q["learned"] - q["proxy"] for q in res])
    log(f"[quality] mean PSNR {np.mean([q['learned'] for q in res]):.2f} dB, gain over K-truncation "
        f"{gain_t:.2f} dB, over the proxy tail {gain_p:.2f} dB")
    assert gain_t >= GAIN_TRUNC_MIN and gain_p >= GAIN_PROXY_MIN
