"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare it with the FP64 oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

RGBA_TOL = 1e-4  # per channel


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_renderer(mesh, workspace_bytes=1 << 28, tuning=None):
    import paper_2009_06574_amd as hx
    r = hx.Renderer(0)
    r.set_workspace(workspace_bytes)
    if tuning is not None:
        r.set_tuning(*tuning)
    r.upload(mesh)
    return r


def gpu_lists(r, cam):
    """Build on the GPU; return (counts u32 [P], off u64 [P+1], rec u64 [F]) row-major."""
    import torch
    r.build(cam)
    c, o, rec = r.export_sorted_lists()
    torch.cuda.synchronize()
    c = c.cpu().numpy().view(np.uint32)
    o = o.cpu().numpy().view(np.uint64)
    rec = rec.cpu().numpy().view(np.uint64)
    return c, o, rec


def rgba_mismatch(gpu, ref, ncand, cand_off, cand, tol=RGBA_TOL):
    """Indices of pixels where the GPU value is within `tol` of neither the
    oracle's nominal result nor any of its alternative results, and the
    indices of pixels the oracle excluded (too many ambiguous fragments)."""
    gpu = np.asarray(gpu, dtype=np.float64).reshape(-1, 4)
    ref = np.asarray(ref).reshape(-1, 4)
    d = np.abs(gpu - ref).max(axis=1)
    bad = np.nonzero(d > tol)[0]
    keep = []
    for p in bad:
        if ncand[p] < 0:
            continue
        ok = False
        if ncand[p] > 0:
            alts = cand[cand_off[p]:cand_off[p + 1]]
            ok = bool(np.any(np.abs(alts - gpu[p]).max(axis=1) <= tol))
        if not ok:
            keep.append(p)
    return np.asarray(keep, dtype=np.int64), np.nonzero(ncand < 0)[0]
