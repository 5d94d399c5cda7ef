"""Benchmark: focus+context hex-mesh frames at 1080p on one MI355X.

Workload: a 128^3-cell hex grid through a smooth bend with 5% strongly
sheared 4^3-cell blocks (2,097,152 cells, 6,340,608 faces), 1920x1080, the
16 orbit cameras with their moving spherical hotspots, 8 GB fragment
workspace.  One step = one whole frame (transform, bin, count, scan, fill,
sort + shade + blend) for the next camera.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 32] [--warmup 4] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mesh, cams, hots, styles, row_step: int, single_row_step: int = 24):
    """Time the FP64 oracle (as it stands) on every `row_step`-th row of the
    given views with all its threads, and on every `single_row_step`-th row of
    the first view with one thread."""
    import numpy as np

    import oracle
    om = oracle.Mesh.from_synth(mesh)

    def run(views, step):
        frags, npx, dt = 0, 0, 0.0
        for cam, hot, style in views:
            W, H = cam.width, cam.height
            rows = np.arange(0, H, step)
            pix = (rows[:, None] * W + np.arange(W)[None, :]).ravel().astype(np.int32)
            t0 = time.perf_counter()
            fr = oracle.Frame.from_camera(om, cam, pixels=pix)
            fr.shade(hot, style)
            dt += time.perf_counter() - t0
            frags += fr.nfrag
            npx += pix.size
        return frags, npx, dt

    views = list(zip(cams, hots, styles))
    threads = oracle.num_threads()
    frags, npx, dt = run(views, row_step)
    oracle.set_num_threads(1)
    f1, n1, d1 = run(views[:1], single_row_step)
    oracle.set_num_threads(threads)
    return dict(value=frags / dt, unit="fragments/s", cores=threads, kind="oracle", cpu_model=cpu_model(),
                sample=f"views 0-{len(cams) - 1}, every {row_step}th row ({npx} pixels, {frags} fragments), "
                       f"{dt:.1f} s of raster + sort + shade + blend; mesh attribute preprocessing excluded",
                single_thread=dict(value=f1 / d1, unit="fragments/s", cores=1,
                                   sample=f"view 0, every {single_row_step}th row ({n1} pixels, {f1} fragments), "
                                          f"{d1:.1f} s"),
                seconds=dt)


# kernel symbols of the timed entries (rocprofv3 names)
KERNEL_SYMBOL = {"fill": "hexfc::k_fill<8, 8>", "count": "hexfc::k_count<8, 8>", "resolve_c0": "k_resolve_short<16>",
                 "resolve_c1": "k_resolve_wave<1>", "resolve_c2": "k_resolve_wave<2>",
                 "resolve_c3": "k_resolve_wave<4>", "resolve_c4": "k_resolve_wave<8>",
                 "resolve_c5": "k_resolve_wave_wide<16>", "resolve_c6": "k_resolve_wave_wide<32>",
                 "resolve_c7": "hexfc::k_resolve_block", "resolve": "every resolve class kernel, fork to join"}


def measured_traffic(kernel: str):
    """Bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, scaled by the copy calibration; None when there is no
    summary for it or the kernel's sources changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_counters_bent128_1080p.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("traffic "):
            continue
        kv = dict(x.split("=", 1) for x in line.split()[1:])
        if kv.get("kernel") != kernel:
            continue
        # (the kernel's sources, joined by '+', hashed over their concatenation)
        srcs = [os.path.join(ROOT, f) for f in kv["source"].split("+")]
        if not all(os.path.exists(f) for f in srcs):
            return None
        if hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest() != kv["sha256"]:
            return None
        return 1024.0 * (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
                         float(kv["write_kib"]) * float(kv["write_scale"]))
    return None


def batch_views(reps: int = 10):
    """Batched views in one captured graph: 32 random views (1024x1024, one
    hotspot each) of the 64^3 jittered mesh, tile shape and sort switch chosen
    by the autotuner; against the same 32 views rendered one frame at a time."""
    import torch

    import paper_2009_06574_amd as hx
    import synth
    mesh, cams, hots, styles = synth.config3()
    r = hx.Renderer(0)
    r.set_workspace(12 << 30)
    r.upload(mesh)
    choice = r.autotune(cams, hots, styles)
    out = torch.empty((len(cams), cams[0].height, cams[0].width, 4), dtype=torch.float32, device="cuda")
    for _ in range(2):
        r.render_batch(cams, hots, styles, out=out)
    frags, overflow = r.batch_status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r.render_batch(cams, hots, styles, out=out)
    torch.cuda.synchronize()
    ms_batch = 1000.0 * (time.perf_counter() - t0) / reps
    single = torch.empty((cams[0].height, cams[0].width, 4), dtype=torch.float32, device="cuda")
    for i in range(2):
        r.render(cams[i], hots[i], styles[i], out=single)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, h, st in zip(cams, hots, styles):
        r.render(c, h, st, out=single)
    torch.cuda.synchronize()
    ms_single = 1000.0 * (time.perf_counter() - t0)
    log(f"[bench] batch of {len(cams)} views: {ms_batch:.2f} ms ({frags / ms_batch / 1e6:.2f} G fragments/s), "
        f"one at a time {ms_single:.2f} ms, tuning {choice}")
    return dict(workload=f"64^3 jittered hex grid, {len(cams)} random views at 1024x1024, one graph launch",
                tuning=dict(tile_w=choice[0], tile_h=choice[1], t_sort=choice[2]),
                ms_per_batch=round(ms_batch, 3), fragments_per_batch=int(frags), overflow=bool(overflow),
                fragments_per_s=frags / ms_batch * 1e3, ms_views_one_at_a_time=round(ms_single, 3),
                speedup_vs_one_at_a_time=round(ms_single / ms_batch, 3))


def learned_tail(r, mesh, conf_min, seeds=range(1001, 1017)):
    """Exact vs learned-tail resolve on the same lists: held-out random views
    of the benchmark mesh (the network was trained on seeds 1-1000)."""
    import numpy as np
    import torch

    from paper_2009_06574_amd import tail
    p_np, meta = tail.load_weights()
    params = torch.tensor(p_np, device="cuda")
    res = []
    for cam, hot, st in tail._views(mesh, seeds, 1920, 1080):
        d = tail.evaluate_view(r, cam, hot, st, params, meta["K"], (conf_min,), reps=5)
        res.append(d)
        lv = d["learned"][str(conf_min)]
        log(f"[bench] learned tail: exact {d['ms_exact']:.3f} ms, learned {lv['ms']:.3f} ms, "
            f"PSNR {lv['psnr']:.2f} dB, fallback {lv['fallback_pixels']} of {d['long_pixels']} long pixels")
    L = [d["learned"][str(conf_min)] for d in res]
    ms_e = float(np.mean([d["ms_exact"] for d in res]))
    ms_l = float(np.mean([x["ms"] for x in L]))
    return dict(K=meta["K"], conf_min=conf_min, views=f"held-out random views, seeds {seeds[0]}-{seeds[-1]}",
                resolve_exact_ms=round(ms_e, 4), resolve_learned_ms=round(ms_l, 4), speedup=round(ms_e / ms_l, 3),
                psnr_db_mean=round(float(np.mean([x["psnr"] for x in L])), 2),
                psnr_db_min=round(float(min(x["psnr"] for x in L)), 2),
                fallback_frac=round(float(np.sum([x["fallback_pixels"] for x in L]) /
                                          max(1, np.sum([d["long_pixels"] for d in res]))), 4),
                head_opaque_frac=round(float(np.mean([d["head_opaque_frac"] for d in res])), 4),
                approx_baselines={k: dict(psnr_db=round(float(np.mean([d["approx"][k]["psnr"] for d in res])), 2),
                                          resolve_ms=round(float(np.mean([d["approx"][k]["ms"] for d in res])), 4))
                                  for k in res[0]["approx"]},
                psnr_db_k_truncation=round(float(np.mean([d["psnr_truncated"] for d in res])), 2),
                psnr_db_proxy_tail=round(float(np.mean([d["psnr_proxy"] for d in res])), 2))


def lod_build(mesh, threads: int = 16):
    """Time the library's sheet-based LoD builder (host C++) on the benchmark
    mesh; its topology is the 128^3 grid, whose hierarchy is the dyadic one
    the synthetic levels already hold (checked)."""
    import numpy as np

    import paper_2009_06574_amd as hx
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        levels, info = hx.build_lod(mesh.hex, mesh.V, threads)
        ts.append(time.perf_counter() - t0)
    same = bool(np.array_equal(levels, mesh.cell_edge_level))
    log(f"[bench] LoD build {min(ts):.2f} s on {threads} threads ({info['sheets']} sheets, "
        f"{info['levels']} levels, equals the mesh's levels: {same})")
    return {"seconds": round(min(ts), 3), "threads": threads, "cells": mesh.C, "sheets": info["sheets"],
            "levels": info["levels"], "merges": info["merges"], "equals_mesh_levels": same,
            "paper_context": "cubic128 (2,097,152 cells): 23.0 s on a Ryzen 9 3900X (Table 1), other CPU"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-row-step", type=int, default=1)
    ap.add_argument("--cpu-views", type=int, default=3, help="views timed for the CPU oracle baseline")
    ap.add_argument("--grid", type=int, default=128, help="grid size (128 = the benchmark workload)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-tail resolve comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-views measurement")
    ap.add_argument("--no-lod", action="store_true", help="skip the LoD-build timing")
    ap.add_argument("--conf-min", type=float, default=0.6,
                    help="learned tail: pixel confidence threshold (0.6: at least 45 dB on every held-out view)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 4 plain device copies of MIB MiB (scale for HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the screen-space split across GPUs is described, not built)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 4, "read_kib": n / 1024, "write_kib": n / 1024}))
        return

    import numpy as np
    import torch

    import paper_2009_06574_amd as hx
    import synth

    hx.load()
    t0 = time.perf_counter()
    if args.grid == 128:
        mesh, cams, hots, styles = synth.config2()
    else:
        mesh, cams, hots, styles = synth.scaled_config(args.grid, 1920, 1080, "bent")
    log(f"[bench] mesh {mesh.name}: {mesh.V} vertices, {mesh.C} cells ({time.perf_counter() - t0:.1f} s)")
    r = hx.Renderer(0)
    r.set_workspace(8 << 30)
    t0 = time.perf_counter()
    r.upload(mesh)
    log(f"[bench] upload {time.perf_counter() - t0:.1f} s")
    out = torch.empty((1080, 1920, 4), dtype=torch.float32, device="cuda")
    nv = len(cams)
    # Statistics of each view (fragments, bin entries, per-class sizes): one
    # frame per view, read back; the timed frames below read nothing back
    # (render_frame neither waits nor copies), so fragments/s counts the
    # known fragments of the views rendered.
    view_stats = []
    for k in range(nv):
        r.render(cams[k], hots[k], styles[k], out=out)
        view_stats.append(r.frame_stats())
    for i in range(args.warmup):
        r.render(cams[i % nv], hots[i % nv], styles[i % nv], out=out)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({nv} sizing + {args.warmup} frames)")
    for k, st in enumerate(view_stats):
        log(f"[bench] view {k}: {st['fragments']} fragments, classes {st['classes']}")
    seq = [(args.warmup + i) % nv for i in range(args.steps)]
    frags = sum(view_stats[k]["fragments"] for k in seq)
    bins = sum(view_stats[k]["bins"] for k in seq)
    # the clean timing: no per-launch events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in seq:
        r.render(cams[k], hots[k], styles[k], out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fl, over = r.batch_status()
    assert not over, "a timed frame outgrew its sizes"
    ms_frame = 1000.0 * dt / args.steps
    log(f"[bench] {args.steps} frames in {dt:.3f} s: {ms_frame:.3f} ms/frame, {frags / dt / 1e9:.3f} G fragments/s")
    # the same frames again with HIP events around every launch (per-kernel times)
    r.set_profiling(True)
    r.kernel_times()
    for k in seq:
        r.render(cams[k], hots[k], styles[k], out=out)
    torch.cuda.synchronize()
    kt = r.kernel_times()
    r.set_profiling(False)

    # rooflines of single kernels from the HIP events recorded around their
    # launches on their own streams: the fill (8 B per fragment written, 4 B
    # per bin entry and 8 B of offsets per pixel read), the coverage count
    # (4 B per bin entry read, 4 B per pixel written) and the resolve kernel
    # of each length class c (8 B per fragment of the class read, 32 B per
    # pixel of the class: count, offsets, RGBA); and of the whole resolve (all
    # classes, both streams, fork to join) for reference
    P = 1920 * 1080
    cls_frags = [sum(view_stats[k]["class_fragments"][c] for k in seq) for c in range(8)]
    cls_pix = [sum(view_stats[k]["classes"][c] for k in seq) for c in range(8)]
    alg = {"fill": 8.0 * frags + 4.0 * bins + 8.0 * P * args.steps,
           "count": 4.0 * bins + 4.0 * P * args.steps,
           "resolve": 8.0 * frags + 32.0 * P * args.steps}
    for c in range(8):
        alg[f"resolve_c{c}"] = 8.0 * cls_frags[c] + 32.0 * cls_pix[c]
    rooflines = {}
    for k, b in alg.items():
        if k not in kt:
            continue
        ms_k, n_k = kt[k]
        ach = (b / n_k) / (ms_k / n_k * 1e-3) / 1e9
        traffic = measured_traffic(k) if args.grid == 128 else None
        rooflines[k] = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                            frac=round(ach / HBM_PEAK_GBS, 4), traffic=None if traffic is None else int(traffic),
                            kernel=KERNEL_SYMBOL.get(k, k), avg_launch_ms=round(ms_k / n_k, 4),
                            bytes_per_launch=int(b / n_k))
    # the dominant kernel: of the single kernels on the render stream (the
    # coverage count, the fill, the resolve of classes 0-3; classes 4-7 run on
    # a second stream and their event times include waiting), the one with the
    # longest time per frame
    singles = [k for k in ("count", "fill", "resolve_c0", "resolve_c1", "resolve_c2", "resolve_c3") if k in rooflines]
    dom = max(singles, key=lambda k: kt[k][0])
    roofline = dict(rooflines[dom])
    roofline["others"] = {k: {x: v[x] for x in ("kernel", "achieved", "frac", "avg_launch_ms", "bytes_per_launch",
                                                "traffic")}
                          for k, v in rooflines.items() if k != dom}
    kernel_ms = {k: round(v[0] / args.steps, 4) for k, v in kt.items()}
    top = {k: v for k, v in kernel_ms.items() if not k.startswith("resolve_c")}
    log(f"[bench] per-frame kernel ms: {top} (sum {sum(top.values()):.3f})")
    log(f"[bench] resolve by class, ms per frame: "
        f"{ {k: v for k, v in kernel_ms.items() if k.startswith('resolve_c')} }")
    for k, v in rooflines.items():
        log(f"[bench] {k}: {v['achieved']:.1f} GB/s ({v['frac']:.1%} of HBM peak), {v['avg_launch_ms']:.4f} ms")

    learned = None
    if not args.no_learned:
        learned = learned_tail(r, mesh, args.conf_min)
    r.close()
    r.workspace = None
    torch.cuda.empty_cache()
    batch = None
    if not args.no_batch:
        batch = batch_views()

    lod = None if args.no_lod else lod_build(mesh)

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline ...")
        cpu = cpu_baseline(mesh, cams[:args.cpu_views], hots[:args.cpu_views], styles[:args.cpu_views],
                           args.cpu_row_step)
        log(f"[bench] oracle {cpu['value'] / 1e6:.2f} M fragments/s on {cpu['cores']} threads ({cpu['seconds']:.1f} s), "
            f"{cpu['single_thread']['value'] / 1e6:.2f} M fragments/s on one thread; {cpu['cpu_model']}")
        cpu.pop("seconds")

    line = {
        "metric": "ms/frame & fragments/s at 1080p; exact vs learned-tail resolve at >=45 dB PSNR",
        "value": frags / dt,
        "unit": "fragments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_frame,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"bent+sheared {args.grid}^3 hex grid, 1920x1080, 16 orbit views, exact resolve",
                   "cells": mesh.C, "faces": 3 * args.grid * args.grid * (args.grid + 1),
                   "fragments_per_frame": frags / args.steps, "workspace_GB": 8},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned_tail": learned,
        "batch": batch,
        "lod_build": lod,
        "detail": {"kernel_ms_per_frame": kernel_ms,
                   "paper_context": "cubic128 (2,097,152 cells) at 1920x1080 on an RTX 2070 SUPER: "
                                    "147.3 ms/frame (45.8 F+C + 101.5 PPFL), other mesh and hardware"},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
