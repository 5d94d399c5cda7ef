"""Independent FP64 world-space ray casting used to pin the oracle.

Nothing here is shared with the oracle or the HIP path: pixel rays are built
by inverting the float camera matrix, and triangles are intersected in world
space (Moller-Trumbore).  The oracle instead snaps vertices to an integer
screen grid and tests edge functions, so agreement away from the snap band is
an independent check of its coverage, fill rule and depth order.
"""
from __future__ import annotations

import numpy as np

# VTK hexahedron faces (same public convention the renderer's input uses)
FACES = [(0, 4, 7, 3), (1, 2, 6, 5), (0, 1, 5, 4), (3, 7, 6, 2), (0, 3, 2, 1), (4, 5, 6, 7)]


def unique_faces(hexes):
    """Faces of a hex mesh, deduplicated in first-seen order (corner order of
    the first cell that has the face)."""
    seen = {}
    out = []
    for c in range(hexes.shape[0]):
        for f in FACES:
            vs = tuple(int(hexes[c, k]) for k in f)
            key = tuple(sorted(vs))
            if key not in seen:
                seen[key] = len(out)
                out.append(vs)
    return np.asarray(out, dtype=np.int64).reshape(-1, 4)


def pixel_rays(view_proj, W, H):
    """Eye position and unit direction of every pixel-centre ray (row-major)."""
    M = np.asarray(view_proj, dtype=np.float64).reshape(4, 4)
    A = np.stack([M[0], M[1], M[3]])
    eye = np.linalg.solve(A[:, :3], -A[:, 3])
    i = np.arange(W) + 0.5
    j = np.arange(H) + 0.5
    nx = 2 * i / W - 1
    ny = 1 - 2 * j / H
    NX, NY = np.meshgrid(nx, ny)
    NX, NY = NX.ravel(), NY.ravel()
    dirs = np.empty((NX.size, 3))
    for p in range(NX.size):
        B = np.stack([M[0] - NX[p] * M[3], M[1] - NY[p] * M[3], M[3]])
        X1 = np.linalg.solve(B[:, :3], np.array([0.0, 0.0, 1.0]) - B[:, 3])
        d = X1 - eye
        dirs[p] = d / np.linalg.norm(d)
    return eye, dirs


def project(view_proj, W, H, P):
    """FP64 screen positions in sub-pixel units (16 per pixel, y down)."""
    M = np.asarray(view_proj, dtype=np.float64).reshape(4, 4)
    Ph = np.concatenate([P, np.ones((P.shape[0], 1))], axis=1)
    c = Ph @ M.T
    x = (c[:, 0] / c[:, 3] + 1) * 0.5 * W * 16
    y = (1 - c[:, 1] / c[:, 3]) * 0.5 * H * 16
    return np.stack([x, y], axis=1), c[:, 3]


def seg_dist2d(px, py, a, b):
    ab = b - a
    l2 = ab @ ab
    t = np.clip(((px - a[0]) * ab[0] + (py - a[1]) * ab[1]) / max(l2, 1e-300), 0, 1)
    dx = px - (a[0] + t * ab[0])
    dy = py - (a[1] + t * ab[1])
    return np.sqrt(dx * dx + dy * dy)


def raycast(P, tris, view_proj, W, H, band=1.0):
    """World-space hits of every pixel ray.

    Returns (hits, near) where hits[p] is a list of (t, tri_id) and near[p] is
    True when a projected triangle edge passes within ``band`` sub-pixels of
    the pixel centre (where snapping may legitimately change coverage)."""
    eye, dirs = pixel_rays(view_proj, W, H)
    S, w = project(view_proj, W, H, P)
    npx = W * H
    hits = [[] for _ in range(npx)]
    near = np.zeros(npx, dtype=bool)
    pxc = (np.arange(npx) % W) * 16 + 8.0
    pyc = (np.arange(npx) // W) * 16 + 8.0
    for tid, (a, b, c) in enumerate(tris):
        if min(w[a], w[b], w[c]) <= 1.0 / 16:
            continue
        xs = S[[a, b, c], 0]
        ys = S[[a, b, c], 1]
        i0 = max(int(np.floor((xs.min() - 8 - 2 * band) / 16)), 0)
        i1 = min(int(np.ceil((xs.max() - 8 + 2 * band) / 16)), W - 1)
        j0 = max(int(np.floor((ys.min() - 8 - 2 * band) / 16)), 0)
        j1 = min(int(np.ceil((ys.max() - 8 + 2 * band) / 16)), H - 1)
        if i0 > i1 or j0 > j1:
            continue
        ii, jj = np.meshgrid(np.arange(i0, i1 + 1), np.arange(j0, j1 + 1))
        pid = (jj * W + ii).ravel()
        px, py = pxc[pid], pyc[pid]
        for u, v in ((a, b), (b, c), (c, a)):
            dd = seg_dist2d(px, py, S[u], S[v])
            near[pid[dd < band]] = True
        # Moller-Trumbore in world space
        v0, v1, v2 = P[a], P[b], P[c]
        e1, e2 = v1 - v0, v2 - v0
        D = dirs[pid]
        pvec = np.cross(D, e2)
        det = pvec @ e1
        ok = np.abs(det) > 1e-300
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        tvec = eye - v0
        uu = (pvec @ tvec) * inv
        qvec = np.cross(tvec, e1)
        vv = (D * qvec).sum(axis=1) * inv
        tt = (qvec @ e2) * inv
        inside = ok & (uu >= 0) & (vv >= 0) & (uu + vv <= 1) & (tt > 0)
        for p, t in zip(pid[inside], tt[inside]):
            hits[p].append((float(t), tid))
    return hits, near
