"""Learned tail compositor: training data, training and evaluation.

Everything numeric runs in the library's HIP kernels through the C ABI:
``hexfc_build_fragment_lists`` and ``hexfc_learned_features`` generate the
training rows (head composite, 9 tail features, exact tail composite),
``hexfc_mlp_forward`` / ``hexfc_mlp_loss`` / ``hexfc_mlp_backward`` /
``hexfc_mlp_adam_step`` train the network, ``hexfc_resolve_learned`` and
``hexfc_resolve`` are compared for quality (PSNR) and speed.  PyTorch only
holds device buffers, draws minibatch indices and times with events.

The learned tail is not part of the paper's method: it follows the paper's
future-work remark on approximating order-independent transparency
(Section 8), with the exact sort-and-blend resolve as its fallback and as the
reference its quality is measured against.

Command line (runs on a GPU)::

    python -m paper_2009_06574_amd.tail train --out weights.npz
    python -m paper_2009_06574_amd.tail eval --weights weights.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import Renderer, mlp_adam_step, mlp_backward, mlp_forward, mlp_loss, mlp_param_count

NF, NH, NO = 9, 64, 5
_SIZES = (("mu", NF), ("inv_sigma", NF), ("W1", NF * NH), ("b1", NH), ("W2", NH * NH), ("b2", NH),
          ("W3", NH * NO), ("b3", NO))
OFF = {}
_o = 0
for _k, _n in _SIZES:
    OFF[_k] = (_o, _o + _n)
    _o += _n
PARAM_COUNT = _o
FEATURES = ("log1p_tail_len", "alpha_sum", "z_mean", "z2_mean", "proxy_r", "proxy_g", "proxy_b", "proxy_a",
            "z_first")
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "tail_k8.npz")


def _log(msg):
    print(msg, flush=True)


def init_params(mu, sigma, seed=0) -> np.ndarray:
    """He-style initialisation; the last layer starts small."""
    rng = np.random.default_rng(seed)
    p = np.zeros(PARAM_COUNT, np.float32)
    p[slice(*OFF["mu"])] = mu
    p[slice(*OFF["inv_sigma"])] = 1.0 / np.maximum(np.asarray(sigma, np.float64), 1e-6)
    p[slice(*OFF["W1"])] = rng.normal(0, math.sqrt(2.0 / NF), NF * NH)
    p[slice(*OFF["W2"])] = rng.normal(0, math.sqrt(2.0 / NH), NH * NH)
    p[slice(*OFF["W3"])] = rng.normal(0, math.sqrt(1.0 / NH), NH * NO) * 0.1
    return p


# ---------------------------------------------------------------- data
def sample_rows(rows: dict, K: int, quota: int, gen):
    """Indices of up to `quota` rows with a tail, stratified over log2 of the
    tail length so that long lists are not drowned by short ones."""
    import torch
    nt = torch.round(torch.expm1(rows["feat"][:, 0]))
    keep = nt > 0
    if not bool(keep.any()):
        return torch.zeros(0, dtype=torch.long, device=nt.device)
    b = torch.floor(torch.log2(nt.clamp(min=1)))
    bins = torch.unique(b[keep])
    q = max(1, quota // len(bins))
    out = []
    for bb in bins:
        ids = torch.nonzero(keep & (b == bb)).flatten()
        if ids.numel() > q:
            ids = ids[torch.randperm(ids.numel(), generator=gen, device=ids.device)[:q]]
        out.append(ids)
    return torch.cat(out)


def collect(r: Renderer, views, K: int = 8, per_view: int = 4096, seed: int = 0, label=""):
    """Training rows (features [n, 9], exact tail targets [n, 4]) from a list
    of (camera, hotspot, style) views of the uploaded mesh."""
    import torch
    gen = torch.Generator(device=r.device)
    gen.manual_seed(seed)
    feats, targets = [], []
    t0 = time.time()
    for i, (cam, hot, st) in enumerate(views):
        r.build(cam)
        rows = r.learned_features(hot, st, K, with_target=True)
        idx = sample_rows(rows, K, per_view, gen)
        feats.append(rows["feat"][idx])
        targets.append(rows["target"][idx])
        if (i + 1) % 100 == 0 or i + 1 == len(views):
            _log(f"[tail] {label} collected {i + 1}/{len(views)} views, "
                 f"{sum(int(f.shape[0]) for f in feats)} rows, {time.time() - t0:.1f} s")
    return torch.cat(feats), torch.cat(targets)


# ---------------------------------------------------------------- training
def train(feat, target, steps: int = 20000, batch: int = 8192, lr: float = 2e-3, lr_end: float = 2e-5,
          seed: int = 0, log_every: int = 1000, conf_tol: float = 0.02):
    """Adam on the mean loss (MSE on the tail RGBA + 0.1 BCE on the
    confidence), with a cosine learning-rate decay.  Returns the FP32
    parameter tensor and the loss history."""
    import torch
    dev = feat.device
    mu = feat.mean(0).double().cpu().numpy()
    sd = feat.std(0).double().cpu().numpy()
    p = torch.tensor(init_params(mu, sd, seed), device=dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    g = torch.zeros_like(p)
    n = feat.shape[0]
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed + 1)
    hist = []
    loss_acc = torch.zeros(1, device=dev)
    t0 = time.time()
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (batch,), generator=gen, device=dev)
        x, t = feat[idx].contiguous(), target[idx].contiguous()
        y = mlp_forward(p, x)
        dy, _ = mlp_loss(y, t, loss_sum=loss_acc, conf_tol=conf_tol)
        g.zero_()
        mlp_backward(p, x, dy, grad=g)
        cur = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * (step - 1) / max(steps - 1, 1)))
        mlp_adam_step(p, m, v, g, step, lr=cur)
        if step % log_every == 0 or step == steps:
            l = float(loss_acc.item()) / (batch * (log_every if step % log_every == 0 else step % log_every))
            loss_acc.zero_()
            hist.append((step, l))
            _log(f"[tail] step {step}/{steps} loss {l:.3e} lr {cur:.2e} ({time.time() - t0:.1f} s)")
    return p, hist


def tail_error(p, feat, target):
    """Max-channel absolute error of the predicted tail and the predicted confidence."""
    import torch
    y = mlp_forward(p, feat)
    err = (y[:, :4].clamp(0, 1) - target).abs().max(dim=1).values
    conf = torch.sigmoid(y[:, 4])
    return err, conf


# ---------------------------------------------------------------- evaluation
def psnr(a, b) -> float:
    mse = float(((a - b) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def baselines(r: Renderer, hot, st, K, exact):
    """Images of two learning-free tails for comparison: K-truncation (the
    tail is dropped) and the proxy tail itself (the ordered composite of the
    proxy shading, features f4..f7)."""
    import torch
    rows = r.learned_features(hot, st, K)
    f = rows["feat"]
    h = rows["head"]
    bg = torch.tensor(list(st.bg) + [0.0], device=h.device)
    pix = rows["pix"].long()
    keep = f[:, 0] > 0  # lists longer than K
    out = {}
    for name, tail in (("truncated", torch.zeros_like(h)), ("proxy", f[:, 4:8])):
        comp = h + (1 - h[:, 3:4]) * tail
        comp = comp + (1 - comp[:, 3:4]) * bg
        img = exact.clone().reshape(-1, 4)
        img[pix[keep]] = comp[keep]
        out[name] = img.reshape(exact.shape)
    return out


def time_call(fn, reps: int = 5) -> float:
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    ts = []
    for _ in range(reps):
        e0.record(s)
        fn()
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def evaluate_view(r: Renderer, cam, hot, st, params, K=8, conf_mins=(0.5,), reps=5) -> dict:
    """Exact vs learned resolve of one view: PSNR (RGB of the final image),
    resolve times, fallback counts, for each confidence threshold."""
    import torch
    r.build(cam)
    exact = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=r.device)
    learned = torch.empty_like(exact)
    mask = torch.empty((cam.height, cam.width), dtype=torch.uint8, device=r.device)
    t_exact = time_call(lambda: r.resolve(hot, st, out=exact), reps)
    base = baselines(r, hot, st, K, exact)
    rgb = slice(0, 3)
    stats = r.frame_stats()
    rows = r.learned_features(hot, st, K)
    eps = 2.0 ** -20
    head_opaque = float(((1 - rows["head"][:, 3]) < eps).float().mean()) if rows["head"].shape[0] else 0.0
    out = dict(ms_exact=t_exact, long_pixels=sum(stats["classes"][1:7]), fragments=stats["fragments"],
               head_opaque_frac=head_opaque,
               psnr_truncated=psnr(base["truncated"][..., rgb], exact[..., rgb]),
               psnr_proxy=psnr(base["proxy"][..., rgb], exact[..., rgb]), learned={})
    # non-learned order-independent approximations on the same lists
    out["approx"] = {}
    for name, method, kk in (("mlab4", "mlab", 4), ("mlab8", "mlab", 8), ("moments", "moments", 0)):
        t_a = time_call(lambda: r.resolve_approx(hot, st, method, kk, out=learned), reps)
        out["approx"][name] = dict(psnr=psnr(learned[..., rgb], exact[..., rgb]), ms=t_a)
    for cm in conf_mins:
        t_l = time_call(lambda: r.resolve_learned(hot, st, params, K, cm, out=learned, mask=mask), reps)
        r.batch_status()
        fb = sum(r.frame_stats()["fallback"])
        out["learned"][str(cm)] = dict(psnr=psnr(learned[..., rgb], exact[..., rgb]), psnr_rgba=psnr(learned, exact),
                                       ms=t_l, speedup=t_exact / t_l, fallback_pixels=fb,
                                       learned_pixels=int((mask == 0).sum()))
    r.set_profiling(True)
    r.kernel_times()
    r.resolve(hot, st, out=exact)
    out["kernels_exact"] = {k: round(v[0], 4) for k, v in r.kernel_times().items()}
    r.resolve_learned(hot, st, params, K, conf_mins[-1], out=learned, mask=mask)
    out["kernels_learned"] = {k: round(v[0], 4) for k, v in r.kernel_times().items()}
    r.set_profiling(False)
    return out


def load_weights(path=DEFAULT_WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        p = np.asarray(z["params"], np.float32)
        meta = json.loads(str(z["meta"]))
    if p.size != mlp_param_count():
        raise ValueError(f"{path}: {p.size} parameters, expected {mlp_param_count()}")
    return p, meta


def save_weights(path, params, meta):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=np.asarray(params, np.float32), meta=np.array(json.dumps(meta)))


# ---------------------------------------------------------------- command line
def _views(mesh, seeds, W, H):
    import synth
    out = []
    for s in seeds:
        c, h, st = synth.random_views(mesh, 1, W, H, seed=s)
        out.append((c[0], h[0], st[0]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--seeds", type=int, default=1000, help="random views per mesh (seeds 1..N)")
    t.add_argument("--per-view", type=int, default=4096)
    t.add_argument("--steps", type=int, default=30000)
    t.add_argument("--batch", type=int, default=8192)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--K", type=int, default=8)
    t.add_argument("--width", type=int, default=1920)
    t.add_argument("--height", type=int, default=1080)
    t.add_argument("--meshes", default="config1,config2")
    t.add_argument("--conf-tol", type=float, default=0.02)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--seeds", default="1001-1016")
    e.add_argument("--conf-min", default="0,0.5,0.8")
    e.add_argument("--width", type=int, default=1920)
    e.add_argument("--height", type=int, default=1080)
    e.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    import torch
    import synth

    r = Renderer(0)
    r.set_workspace(8 << 30)
    if a.cmd == "train":
        feats, targets = [], []
        for name in a.meshes.split(","):
            mesh = getattr(synth, name)()[0]
            r.upload(mesh)
            views = _views(mesh, range(1, a.seeds + 1), a.width, a.height)
            f, tt = collect(r, views, a.K, a.per_view, seed=len(feats), label=name)
            feats.append(f)
            targets.append(tt)
        feat, target = torch.cat(feats), torch.cat(targets)
        _log(f"[tail] {feat.shape[0]} training rows")
        p, hist = train(feat, target, a.steps, a.batch, a.lr, conf_tol=a.conf_tol)
        err, conf = tail_error(p, feat[:200000], target[:200000])
        meta = dict(K=a.K, features=FEATURES, rows=int(feat.shape[0]), steps=a.steps, batch=a.batch, lr=a.lr,
                    conf_tol=a.conf_tol,
                    meshes=a.meshes, seeds=[1, a.seeds], per_view=a.per_view, final_loss=hist[-1][1],
                    train_err_median=float(err.median()), train_err_p99=float(err.quantile(0.99)),
                    train_frac_within_tol=float((err < a.conf_tol).float().mean()),
                    train_conf_mean=float(conf.mean()))
        save_weights(a.out, p.cpu().numpy(), meta)
        _log(f"[tail] saved {a.out}: {json.dumps(meta)}")
        return 0
    p_np, meta = load_weights(a.weights)
    params = torch.tensor(p_np, device=r.device)
    mesh = synth.config2()[0]
    r.upload(mesh)
    lo, hi = (int(x) for x in a.seeds.split("-"))
    cms = tuple(float(x) for x in a.conf_min.split(","))
    res = []
    for s, (cam, hot, st) in zip(range(lo, hi + 1), _views(mesh, range(lo, hi + 1), a.width, a.height)):
        d = evaluate_view(r, cam, hot, st, params, meta["K"], cms)
        d["seed"] = s
        res.append(d)
        _log("[tail] " + json.dumps(d))
    summary = {k: float(np.mean([d[k] for d in res])) for k in ("ms_exact", "psnr_truncated", "psnr_proxy")}
    for cm in cms:
        for k in ("psnr", "ms", "speedup", "fallback_pixels", "learned_pixels"):
            summary[f"{k}@{cm}"] = float(np.mean([d["learned"][str(cm)][k] for d in res]))
        summary[f"psnr_min@{cm}"] = float(min(d["learned"][str(cm)]["psnr"] for d in res))
    _log("[tail] mean " + json.dumps(summary))
    if a.json:
        with open(a.json, "w") as f:
            json.dump(dict(views=res, mean=summary, weights=os.path.basename(a.weights)), f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
