"""Seeded synthetic inputs for the focus+context hex-mesh renderer.

This module only *generates inputs*: structured hex grids with jitter, bends and
sheared blocks, perspective cameras, spherical hotspots, style parameters and a
dyadic stand-in for the per-edge LoD levels.  It holds none of the rendering
method's arithmetic (no quantisation, no Jacobians, no rasterisation, no
shading), so both the HIP library and the CPU oracle may consume it.

The paper's meshes (fandisk ... cubic128, Section 7, Table 1) are not
available; the grids below stand in for them with the sizes and depth
complexity of its largest data set (a 128^3 Cartesian grid).

Conventions
-----------
* Vertex (i, j, k) of an N^3 grid has index ``i + (N+1)*(j + (N+1)*k)`` and
  rest position ``(i, j, k) / N``.
* Cell (i, j, k) has index ``i + N*(j + N*k)``; its 8 corners follow the VTK
  hexahedron order: 0=(i,j,k) 1=(i+1,j,k) 2=(i+1,j+1,k) 3=(i,j+1,k), 4..7 the
  same at k+1.
* Local cell edges (the layout of ``cell_edge_level[C][12]``):
  0:(0,1) 1:(1,2) 2:(2,3) 3:(3,0) 4:(4,5) 5:(5,6) 6:(6,7) 7:(7,4)
  8:(0,4) 9:(1,5) 10:(2,6) 11:(3,7).
* Cameras are row-major float32 world->clip matrices (OpenGL-style
  perspective, clip w = distance along the view axis), plus width/height.
* All randomness uses ``numpy.random.default_rng(seed)`` (PCG64) with the
  draw order stated in each generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CELL_EDGES = np.array(
    [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4),
     (0, 4), (1, 5), (2, 6), (3, 7)], dtype=np.int32)

# corner offsets (di, dj, dk) of the 8 VTK-ordered hexahedron corners
_CORNER_OFF = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                        (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)], dtype=np.int64)


@dataclass
class Mesh:
    """A hexahedral mesh as handed to the renderer (host arrays)."""
    xyz: np.ndarray              # float32 [V, 3]
    hex: np.ndarray              # int32   [C, 8] VTK corner order
    cell_edge_level: np.ndarray  # uint8   [C, 12] (local edge table above)
    cell_scalar: np.ndarray | None = None   # float32 [C] or None (-> 1 - scaled Jacobian)
    name: str = ""

    @property
    def V(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def C(self) -> int:
        return int(self.hex.shape[0])

    def bbox(self):
        return self.xyz.min(axis=0).astype(np.float64), self.xyz.max(axis=0).astype(np.float64)


@dataclass
class Camera:
    view_proj: np.ndarray        # float32 [4, 4] row-major, world -> clip
    width: int
    height: int
    eye: tuple = (0.0, 0.0, 0.0)
    target: tuple = (0.0, 0.0, 0.0)
    fovy_deg: float = 45.0

    @property
    def distance(self) -> float:
        return float(np.linalg.norm(np.asarray(self.eye) - np.asarray(self.target)))

    def pixel_world(self) -> float:
        """World-space size of one pixel at the camera-to-target distance."""
        return 2.0 * self.distance * math.tan(math.radians(self.fovy_deg) / 2.0) / self.height


@dataclass
class Hotspot:
    center: tuple
    radius: float


@dataclass
class Style:
    """Constant shading parameters (the paper's live-editable shader constants)."""
    w_base: float = 0.0
    k_focus: float = 2.0
    halo_width: float = 0.0
    halo_alpha: float = 1.0
    darken: float = 0.25
    accent_s: float = 1.5
    accent_brighten: float = 0.15
    delta: float = 0.5
    lod: int = 1
    tf_rgb_lo: tuple = (0.0, 0.0, 1.0)
    tf_rgb_hi: tuple = (1.0, 0.0, 0.0)
    tf_a_lo: float = 0.05
    tf_a_hi: float = 0.6
    bg: tuple = (0.0, 0.0, 0.0)
    lens_mode: int = 0          # 0: object-space sphere, 1: screen-space circle (pixels)
    desaturate: float = 0.0     # depth-cue desaturation strength in the focus region
    sil_alpha: float = 0.0      # opacity of the white screen-space silhouettes (0: off)
    sil_tau: float = 0.02       # relative view-depth jump that makes an interior silhouette


# ----------------------------------------------------------------------------- grids

def grid_vertices(N: int) -> np.ndarray:
    """Rest positions (float64 [V,3]) of an N^3-cell grid over [0,1]^3."""
    r = np.arange(N + 1, dtype=np.float64) / N
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


def grid_cells(N: int) -> np.ndarray:
    """Hex connectivity (int32 [N^3, 8]) in VTK corner order."""
    n1 = N + 1
    idx = np.arange(N, dtype=np.int64)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    out = np.empty((i.size, 8), dtype=np.int64)
    for c, (di, dj, dk) in enumerate(_CORNER_OFF):
        out[:, c] = (i + di) + n1 * ((j + dj) + n1 * (k + dk))
    return out.astype(np.int32)


def boundary_vertex_mask(N: int) -> np.ndarray:
    n1 = N + 1
    r = np.arange(n1)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    b = (i == 0) | (i == N) | (j == 0) | (j == N) | (k == 0) | (k == N)
    return b.ravel()


def _ctz(x: np.ndarray) -> np.ndarray:
    out = np.zeros_like(x)
    y = x.copy()
    for _ in range(32):
        m = (y > 0) & ((y & 1) == 0)
        out[m] += 1
        y[m] >>= 1
        if not m.any():
            break
    return out


def dyadic_lod_levels(N: int) -> np.ndarray:
    """Per-cell edge levels (uint8 [C,12]) of the dyadic LoD stand-in.

    Interior grid plane j (0<j<N) has level ctz(j); the two boundary planes of
    each axis have level log2(N).  An edge lies in two axis planes and takes the
    smaller of their levels, so the box's outer edges keep the coarsest level.
    This approximates pairwise merging of adjacent parallel sheets; the real
    sheet-merging hierarchy (Section 5) is preprocessing outside the render path.
    """
    L = int(round(math.log2(N)))
    plane = np.arange(N + 1, dtype=np.int64)
    lev = _ctz(plane)
    lev[0] = L
    lev[N] = L
    idx = np.arange(N, dtype=np.int64)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    out = np.empty((i.size, 12), dtype=np.int64)
    # corner (di,dj,dk) -> edge direction & fixed planes
    for e, (a, b) in enumerate(CELL_EDGES):
        oa, ob = _CORNER_OFF[a], _CORNER_OFF[b]
        axis = int(np.nonzero(oa != ob)[0][0])
        fixed = [ax for ax in range(3) if ax != axis]
        coords = (i, j, k)
        p0 = coords[fixed[0]] + oa[fixed[0]]
        p1 = coords[fixed[1]] + oa[fixed[1]]
        out[:, e] = np.minimum(lev[p0], lev[p1])
    return out.astype(np.uint8)


def jittered_grid(N: int, amp: float = 0.2, seed: int = 0) -> Mesh:
    """N^3 grid over [0,1]^3; every vertex gets U(-amp, amp)/N per axis, then
    the boundary vertices are reset to their rest position.

    Draw order: one ``rng.uniform(-amp, amp, size=(V, 3))`` call.
    """
    rng = np.random.default_rng(seed)
    xyz = grid_vertices(N)
    off = rng.uniform(-amp, amp, size=xyz.shape) / N
    off[boundary_vertex_mask(N)] = 0.0
    xyz = xyz + off
    return Mesh(xyz=xyz.astype(np.float32), hex=grid_cells(N),
                cell_edge_level=dyadic_lod_levels(N), name=f"jitter{N}")


def bent_sheared_grid(N: int = 128, frac: float = 0.05, amp: float = 0.45,
                      block: int = 4, seed: int = 0) -> Mesh:
    """N^3 grid with strongly sheared blocks, mapped through a smooth bend.

    1. Choose ``round(frac * (N/block)^3)`` of the (N/block)^3 blocks of
       block^3 cells without replacement (``rng.choice``).
    2. Draw ``rng.uniform(-amp, amp, size=(V,3))/N``; apply it to every vertex
       of a chosen block that is not on the mesh boundary.
    3. Bend: x' = x, y' = y + 0.3 sin(pi x), z' = z + 0.2 x y.
    """
    rng = np.random.default_rng(seed)
    nb = N // block
    nchoose = int(round(frac * nb ** 3))
    chosen = rng.choice(nb ** 3, size=nchoose, replace=False)
    off = rng.uniform(-amp, amp, size=((N + 1) ** 3, 3)) / N
    n1 = N + 1
    mask = np.zeros((n1, n1, n1), dtype=bool)  # [k, j, i]
    bi = chosen % nb
    bj = (chosen // nb) % nb
    bk = chosen // (nb * nb)
    for a, b, c in zip(bi, bj, bk):
        mask[c * block:(c + 1) * block + 1, b * block:(b + 1) * block + 1,
             a * block:(a + 1) * block + 1] = True
    mask = mask.ravel() & ~boundary_vertex_mask(N)
    xyz = grid_vertices(N)
    xyz[mask] += off[mask]
    x, y, z = xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy()
    xyz[:, 1] = y + 0.3 * np.sin(np.pi * x)
    xyz[:, 2] = z + 0.2 * x * y
    return Mesh(xyz=xyz.astype(np.float32), hex=grid_cells(N),
                cell_edge_level=dyadic_lod_levels(N), name=f"bent{N}")


def box_grid(nx: int, ny: int, nz: int, size=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)) -> Mesh:
    """Axis-aligned nx*ny*nz grid of identical cuboids (no LoD levels set)."""
    xs = origin[0] + np.arange(nx + 1) * (size[0] / nx)
    ys = origin[1] + np.arange(ny + 1) * (size[1] / ny)
    zs = origin[2] + np.arange(nz + 1) * (size[2] / nz)
    k, j, i = np.meshgrid(zs, ys, xs, indexing="ij")
    xyz = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    idx = [np.arange(nx), np.arange(ny), np.arange(nz)]
    kk, jj, ii = np.meshgrid(idx[2], idx[1], idx[0], indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    hexes = np.empty((ii.size, 8), dtype=np.int64)
    for c, (di, dj, dk) in enumerate(_CORNER_OFF):
        hexes[:, c] = (ii + di) + (nx + 1) * ((jj + dj) + (ny + 1) * (kk + dk))
    return Mesh(xyz=xyz.astype(np.float32), hex=hexes.astype(np.int32),
                cell_edge_level=np.zeros((ii.size, 12), dtype=np.uint8), name=f"box{nx}x{ny}x{nz}")



def polygon_prism(k: int, n: int, m: int, twist: float = 0.0, amp: float = 0.0, seed: int = 0) -> Mesh:
    """A k-gon (radius 0.5, centred at (0.5, 0.5)) split into k quads around its
    centre, each quad subdivided n x n, extruded over z in [0, 1] in m layers.

    Block i has corners V_i (polygon corner), M_i (midpoint of side V_i V_i+1),
    the centre O and M_{i-1}; its point (a, b) (0 <= a, b <= n) is the bilinear
    blend of those corners at (a/n, b/n).  For k != 4 the vertical edges through
    the centre are singular (k incident cells); the vertical edges at the polygon
    corners have one incident cell.  Points on the block sides are generated
    once, from the side's end points, so neighbouring blocks share them exactly.

    twist: each layer is rotated by twist * z radians about the prism axis.
    amp: every vertex off the mesh boundary is moved by U(-amp, amp)/n per axis
    (one ``rng.uniform(-amp, amp, size=(V, 3))`` draw).
    Cells are ordered by layer, then block, then b, then a.  No LoD levels set.
    """
    if k < 3 or n < 1 or m < 1:
        raise ValueError("polygon_prism needs k >= 3, n >= 1, m >= 1")
    th = 2.0 * np.pi * np.arange(k) / k
    Vc = np.stack([0.5 * np.cos(th), 0.5 * np.sin(th)], axis=1)
    Mc = 0.5 * (Vc + np.roll(Vc, -1, axis=0))
    O = np.zeros(2)
    keys, pts = {}, []

    def vid(i, a, b):
        """Canonical id of block i's point (a, b)."""
        if a == n and b == n:
            key, p = ("O",), O
        elif a == n:    # side M_i -> O, shared with block i + 1
            key, p = ("I", i, b), Mc[i] + (b / n) * (O - Mc[i])
        elif b == n:    # side M_{i-1} -> O, shared with block i - 1
            j = (i - 1) % k
            key, p = ("I", j, a), Mc[j] + (a / n) * (O - Mc[j])
        elif b == 0:    # polygon side, V_i -> M_i
            key, p = ("S", i, a), Vc[i] + (a / n) * (Mc[i] - Vc[i])
        elif a == 0:    # polygon side, V_i -> M_{i-1}
            j = (i - 1) % k
            key, p = ("T", i, b), Vc[i] + (b / n) * (Mc[j] - Vc[i])
        else:
            u, v = a / n, b / n
            j = (i - 1) % k
            key = ("B", i, a, b)
            p = (1 - u) * (1 - v) * Vc[i] + u * (1 - v) * Mc[i] + u * v * O + (1 - u) * v * Mc[j]
        if key not in keys:
            keys[key] = len(pts)
            pts.append((p, key[0] in ("S", "T")))
        return keys[key]

    quads = []
    for i in range(k):
        for b in range(n):
            for a in range(n):
                quads.append((vid(i, a, b), vid(i, a + 1, b), vid(i, a + 1, b + 1), vid(i, a, b + 1)))
    quads = np.asarray(quads, dtype=np.int64)
    nv2 = len(pts)
    p2 = np.array([p for p, _ in pts])
    side = np.array([s for _, s in pts])
    z = np.arange(m + 1, dtype=np.float64) / m
    ang = twist * z
    ca, sa = np.cos(ang)[:, None], np.sin(ang)[:, None]
    x = ca * p2[None, :, 0] - sa * p2[None, :, 1]
    y = sa * p2[None, :, 0] + ca * p2[None, :, 1]
    xyz = np.stack([0.5 + x, 0.5 + y, np.broadcast_to(z[:, None], x.shape)], axis=2).reshape(-1, 3)
    if amp > 0.0:
        rng = np.random.default_rng(seed)
        off = rng.uniform(-amp, amp, size=xyz.shape) / n
        lay = np.repeat(np.arange(m + 1), nv2)
        bnd = np.tile(side, m + 1) | (lay == 0) | (lay == m)
        off[bnd] = 0.0
        xyz = xyz + off
    L = np.arange(m, dtype=np.int64)[:, None, None]
    hexes = np.concatenate([quads[None] + nv2 * L, quads[None] + nv2 * (L + 1)], axis=2).reshape(-1, 8)
    return Mesh(xyz=xyz.astype(np.float32), hex=hexes.astype(np.int32),
                cell_edge_level=np.zeros((hexes.shape[0], 12), dtype=np.uint8), name=f"prism{k}_{n}x{m}")


# ----------------------------------------------------------------------------- cameras

def look_at(eye, target, up) -> np.ndarray:
    eye, target, up = (np.asarray(v, dtype=np.float64) for v in (eye, target, up))
    f = target - eye
    f = f / np.linalg.norm(f)
    s = np.cross(f, up)
    s = s / np.linalg.norm(s)
    u = np.cross(s, f)
    m = np.eye(4)
    m[0, :3], m[1, :3], m[2, :3] = s, u, -f
    m[0, 3], m[1, 3], m[2, 3] = -s @ eye, -u @ eye, f @ eye
    return m


def perspective(fovy_deg: float, aspect: float, near: float, far: float) -> np.ndarray:
    f = 1.0 / math.tan(math.radians(fovy_deg) / 2.0)
    m = np.zeros((4, 4))
    m[0, 0] = f / aspect
    m[1, 1] = f
    m[2, 2] = (far + near) / (near - far)
    m[2, 3] = 2.0 * far * near / (near - far)
    m[3, 2] = -1.0
    return m


def make_camera(eye, target, width: int, height: int, fovy_deg: float = 45.0,
                up=(0.0, 1.0, 0.0), near: float = 0.1, far: float = 10.0) -> Camera:
    eye = tuple(float(v) for v in eye)
    target = tuple(float(v) for v in target)
    d = np.asarray(target) - np.asarray(eye)
    d = d / np.linalg.norm(d)
    upv = np.asarray(up, dtype=np.float64)
    if abs(float(d @ upv)) > 0.99:
        upv = np.array([0.0, 0.0, 1.0])
    vp = perspective(fovy_deg, width / height, near, far) @ look_at(eye, target, upv)
    return Camera(view_proj=vp.astype(np.float32), width=int(width), height=int(height),
                  eye=eye, target=target, fovy_deg=fovy_deg)


def orbit_camera(target, distance: float, azimuth_deg: float, elevation_deg: float,
                 width: int, height: int, fovy_deg: float = 45.0) -> Camera:
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    dirv = np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    eye = np.asarray(target, dtype=np.float64) + distance * dirv
    return make_camera(eye, target, width, height, fovy_deg)


def default_style(cam: Camera, **over) -> Style:
    """Style of the benchmark configs: 0.5 px base width in context, k=2 (1.5 px in
    focus), halo 0.5*w_base, darken 0.25, s=1.5, brighten 0.15, delta=0.5, lod=1."""
    wb = 0.5 * cam.pixel_world()
    st = Style(w_base=wb, halo_width=0.5 * wb)
    for k, v in over.items():
        setattr(st, k, v)
    return st


# ----------------------------------------------------------------------------- configs

def config0():
    """8^3 jittered grid at 256x256, one camera, hotspot r=0.3 at the center."""
    mesh = jittered_grid(8, 0.2, seed=0)
    cam = orbit_camera((0.5, 0.5, 0.5), 2.5, 30.0, 20.0, 256, 256)
    hot = Hotspot((0.5, 0.5, 0.5), 0.3)
    return mesh, [cam], [hot], [default_style(cam)]


def orbit_views(mesh: Mesh, width: int = 1920, height: int = 1080, n: int = 16, radius: float = 0.15):
    """16 orbit cameras (elevation 20 deg, azimuth k*22.5 deg, distance 2.5) aimed
    at the bbox center; hotspots of radius ``radius`` along the bbox diagonal
    at u_k = 0.1 + 0.8 k/15."""
    lo, hi = mesh.bbox()
    c = 0.5 * (lo + hi)
    cams, hots, styles = [], [], []
    for k in range(n):
        cam = orbit_camera(tuple(c), 2.5, k * 360.0 / n, 20.0, width, height)
        u = 0.1 + 0.8 * k / max(n - 1, 1)
        cams.append(cam)
        hots.append(Hotspot(tuple(lo + u * (hi - lo)), radius))
        styles.append(default_style(cam))
    return cams, hots, styles


def config1():
    mesh = jittered_grid(64, 0.2, seed=0)
    cams, hots, styles = orbit_views(mesh)
    return mesh, cams, hots, styles


def config2():
    mesh = bent_sheared_grid(128, seed=0)
    cams, hots, styles = orbit_views(mesh)
    return mesh, cams, hots, styles


def random_views(mesh: Mesh, n: int, width: int, height: int, seed: int):
    """Random cameras on a sphere (Gaussian direction, radius U(2,3)) aimed at
    the bbox center, with hotspots at U(bbox) of radius U(0.1, 0.3).

    Draw order per view: direction (3 normals), radius, hotspot center (3), radius.
    """
    rng = np.random.default_rng(seed)
    lo, hi = mesh.bbox()
    c = 0.5 * (lo + hi)
    cams, hots, styles = [], [], []
    for _ in range(n):
        d = rng.normal(size=3)
        d = d / np.linalg.norm(d)
        r = rng.uniform(2.0, 3.0)
        hc = lo + rng.uniform(0.0, 1.0, size=3) * (hi - lo)
        hr = rng.uniform(0.1, 0.3)
        cam = make_camera(c + r * d, c, width, height)
        cams.append(cam)
        hots.append(Hotspot(tuple(hc), float(hr)))
        styles.append(default_style(cam))
    return cams, hots, styles


def config3():
    mesh = jittered_grid(64, 0.2, seed=0)
    cams, hots, styles = random_views(mesh, 32, 1024, 1024, seed=0)
    return mesh, cams, hots, styles


def scaled_config(N: int, width: int, height: int, kind: str = "jitter", nviews: int = 16):
    """A smaller stand-in of configs 1/2 (same recipe, grid N^3, given viewport)."""
    mesh = jittered_grid(N, 0.2, 0) if kind == "jitter" else bent_sheared_grid(N, seed=0, block=max(1, min(4, N // 8)))
    cams, hots, styles = orbit_views(mesh, width, height, n=nviews)
    return mesh, cams, hots, styles
