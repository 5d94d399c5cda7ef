"""FP64 CPU oracle of the focus+context hex-mesh render path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product path (the HIP library
and its Python binding) never imports it, and it never imports them.

The arithmetic lives in ``hexfc_oracle.c`` (plain C, FP64, exact integer
geometry); this file only marshals numpy arrays.  Build it with
``oracle.build()`` (gcc, OpenMP).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hexfc_oracle.c")
# HEXFC_ORACLE_LIB: another build of hexfc_oracle.c to load (the sanitizer
# test runs the oracle from an ASan/UBSan build)
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
_LIB = os.environ.get("HEXFC_ORACLE_LIB") or _DEFAULT_LIB
_lib = None

# style vector layout shared with hexfc_oracle.c (ST_* enum)
STYLE_FIELDS = ("w_base", "k_focus", "halo_width", "halo_alpha", "darken", "accent_s",
                "accent_brighten", "delta", "lod")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_DEFAULT_LIB):
        tmp = _DEFAULT_LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _DEFAULT_LIB)
    return _DEFAULT_LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        if _LIB != _DEFAULT_LIB:
            raise OracleError(f"no oracle library at {_LIB}")
        build()
    lib = ct.CDLL(_LIB)
    P = ct.c_void_p
    i64 = ct.c_int64
    lib.orc_mesh_build.argtypes = [P, i64, P, i64, P, P, ct.POINTER(P)]
    lib.orc_mesh_build.restype = ct.c_int
    lib.orc_mesh_free.argtypes = [P]
    lib.orc_mesh_sizes.argtypes = [P, P]
    lib.orc_mesh_export.argtypes = [P, P, P, P, P, P, P]
    lib.orc_mesh_boundary.argtypes = [P, P]
    lib.orc_scaled_jacobian.argtypes = [P]
    lib.orc_scaled_jacobian.restype = ct.c_double
    lib.orc_smoothstep.argtypes = [ct.c_double, ct.c_double, ct.c_double]
    lib.orc_smoothstep.restype = ct.c_double
    lib.orc_set_num_threads.argtypes = [ct.c_int]
    lib.orc_set_num_threads.restype = None
    lib.orc_frame_raster.argtypes = [P, P, ct.c_int, ct.c_int, i64, P, ct.POINTER(P)]
    lib.orc_frame_raster.restype = ct.c_int
    lib.orc_frame_free.argtypes = [P]
    lib.orc_frame_nfrag.argtypes = [P]
    lib.orc_frame_nfrag.restype = i64
    lib.orc_frame_lists.argtypes = [P, P, P, P]
    lib.orc_frame_vertices.argtypes = [P, P, P, P, P]
    lib.orc_frame_shade.argtypes = [P, P, P, P, P]
    lib.orc_frame_shade.restype = ct.c_int
    lib.orc_frame_ncand.argtypes = [P]
    lib.orc_frame_ncand.restype = i64
    lib.orc_frame_cands.argtypes = [P, P, P]
    lib.orc_shade_one.argtypes = [P, i64, i64, ct.c_uint32, P, P, ct.c_uint, P]
    lib.orc_num_threads.restype = ct.c_int
    lib.orc_frame_tail.argtypes = [P, P, P, ct.c_int, ct.c_double, ct.c_double, P, P, P, P]
    lib.orc_frame_tail.restype = ct.c_int
    lib.orc_frame_approx.argtypes = [P, P, P, ct.c_int, ct.c_int, ct.c_double, ct.c_double, ct.c_double,
                                     ct.c_double, P]
    lib.orc_frame_approx.restype = ct.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def style_vector(st) -> np.ndarray:
    """Pack a synth.Style (or anything with the same attributes) into the
    oracle's 24-double style vector."""
    v = [float(getattr(st, k)) for k in STYLE_FIELDS]
    v += [float(x) for x in st.tf_rgb_lo] + [float(x) for x in st.tf_rgb_hi]
    v += [float(st.tf_a_lo), float(st.tf_a_hi)] + [float(x) for x in st.bg]
    v += [float(getattr(st, "lens_mode", 0)), float(getattr(st, "desaturate", 0.0))]
    v += [float(getattr(st, "sil_alpha", 0.0)), float(getattr(st, "sil_tau", 0.02))]
    return np.asarray(v, dtype=np.float64)


def _style(st) -> np.ndarray:
    v = np.ascontiguousarray(style_vector(st) if not isinstance(st, np.ndarray) else st, np.float64)
    if v.shape != (24,):
        raise ValueError("a style vector has 24 entries (see style_vector)")
    return v


def hotspot_vector(h) -> np.ndarray:
    return np.asarray(list(h.center) + [h.radius], dtype=np.float64)


def scaled_jacobian(corners) -> float:
    c = np.ascontiguousarray(np.asarray(corners, dtype=np.float64).reshape(8, 3))
    return float(_load().orc_scaled_jacobian(_ptr(c)))


def smoothstep(e0, e1, x) -> float:
    return float(_load().orc_smoothstep(e0, e1, x))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from here on."""
    _load().orc_set_num_threads(int(n))


# moment-based transparency: bias towards the reference moments and the
# weight of the bound at the fragment's own depth (readings of the method)
MBOIT_BETA = 5e-5
MBOIT_ETA = 0.25


class OracleError(RuntimeError):
    pass


class Mesh:
    """Oracle-side mesh attributes (positions quantised, importance, faces)."""

    def __init__(self, xyz, hex, cell_scalar=None, cell_edge_level=None):
        lib = _load()
        self._xyz = np.ascontiguousarray(xyz, dtype=np.float32)
        self._hex = np.ascontiguousarray(hex, dtype=np.int32)
        self._sc = None if cell_scalar is None else np.ascontiguousarray(cell_scalar, dtype=np.float32)
        self._lv = None if cell_edge_level is None else np.ascontiguousarray(cell_edge_level, dtype=np.uint8)
        h = ct.c_void_p()
        rc = lib.orc_mesh_build(_ptr(self._xyz), self._xyz.shape[0], _ptr(self._hex), self._hex.shape[0],
                                _ptr(self._sc), _ptr(self._lv), ct.byref(h))
        if rc != 0:
            raise OracleError(f"orc_mesh_build failed: {rc}")
        self._h = h
        sizes = np.zeros(3, dtype=np.int64)
        lib.orc_mesh_sizes(h, _ptr(sizes))
        self.V, self.C, self.F = (int(x) for x in sizes)

    @classmethod
    def from_synth(cls, m):
        return cls(m.xyz, m.hex, m.cell_scalar, m.cell_edge_level)

    def boundary(self):
        """uint8 [F]: 1 for faces of one cell only (the mesh boundary surface)."""
        out = np.zeros(self.F, np.uint8)
        _load().orc_mesh_boundary(self._h, _ptr(out))
        return out

    def export(self):
        V, C, F = self.V, self.C, self.F
        out = dict(pos_q=np.zeros((V, 3), np.int32), t_cell=np.zeros(C), t_v=np.zeros(V),
                   face_v=np.zeros((F, 4), np.int32), face_lvl=np.zeros((F, 4), np.uint8),
                   face_te=np.zeros((F, 4)))
        _load().orc_mesh_export(self._h, *(_ptr(out[k]) for k in
                                           ("pos_q", "t_cell", "t_v", "face_v", "face_lvl", "face_te")))
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            _load().orc_mesh_free(self._h)
            self._h = None


class Frame:
    """One camera's exact fragment lists over a set of sample pixels."""

    def __init__(self, mesh: Mesh, view_proj, width: int, height: int, pixels=None):
        lib = _load()
        self.mesh = mesh
        self.W, self.H = int(width), int(height)
        vp = np.ascontiguousarray(np.asarray(view_proj, dtype=np.float32).reshape(16))
        self._pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int32)
        h = ct.c_void_p()
        n = 0 if self._pix is None else self._pix.size
        rc = lib.orc_frame_raster(mesh._h, _ptr(vp), self.W, self.H, n, _ptr(self._pix), ct.byref(h))
        if rc != 0:
            raise OracleError(f"orc_frame_raster failed: {rc}")
        self._h = h
        self.npix = self.W * self.H if self._pix is None else self._pix.size
        self.nfrag = int(lib.orc_frame_nfrag(h))

    @classmethod
    def from_camera(cls, mesh, cam, pixels=None):
        return cls(mesh, cam.view_proj, cam.width, cam.height, pixels)

    def lists(self):
        """(count u32[npix], off u64[npix+1], rec u64[F]) with every list sorted."""
        count = np.zeros(self.npix, np.uint32)
        off = np.zeros(self.npix + 1, np.uint64)
        rec = np.zeros(self.nfrag, np.uint64)
        _load().orc_frame_lists(self._h, _ptr(count), _ptr(off), _ptr(rec))
        return count, off, rec

    def vertices(self):
        V = self.mesh.V
        sx, sy, q = (np.zeros(V, np.int32) for _ in range(3))
        fl = np.zeros(V, np.uint8)
        _load().orc_frame_vertices(self._h, _ptr(sx), _ptr(sy), _ptr(q), _ptr(fl))
        return sx, sy, q, fl

    def shade(self, hotspot, style):
        """FP64 RGBA per sample pixel plus the alternative results of pixels
        whose fragments sit on a discontinuity within FP32 error:
        returns (rgba [npix,4], ncand [npix], cand_off [npix+1], cand [n,4])."""
        lib = _load()
        hv = hotspot_vector(hotspot) if not isinstance(hotspot, np.ndarray) else hotspot
        sv = _style(style)
        hv = np.ascontiguousarray(hv, np.float64)
        rgba = np.zeros((self.npix, 4))
        ncand = np.zeros(self.npix, np.int32)
        rc = lib.orc_frame_shade(self._h, _ptr(hv), _ptr(sv), _ptr(rgba), _ptr(ncand))
        if rc != 0:
            raise OracleError(f"orc_frame_shade failed: {rc}")
        nc = int(lib.orc_frame_ncand(self._h))
        cand_off = np.zeros(self.npix + 1, np.int64)
        cand = np.zeros((nc, 4))
        lib.orc_frame_cands(self._h, _ptr(cand_off), _ptr(cand))
        return rgba, ncand, cand_off, cand

    def shade_one(self, i, j, tri, hotspot, style, flip=0):
        hv = np.ascontiguousarray(hotspot_vector(hotspot) if not isinstance(hotspot, np.ndarray) else hotspot)
        sv = _style(style)
        out = np.zeros(5)
        _load().orc_shade_one(self._h, int(i), int(j), int(tri), _ptr(hv), _ptr(sv), int(flip), _ptr(out))
        return out

    def tail(self, hotspot, style, K, w0, w1):
        """Head composite, tail features and exact tail target per sample pixel
        (learned-tail definition in hexfc_oracle.c): (head, feat, target, has)."""
        hv = np.ascontiguousarray(hotspot_vector(hotspot) if not isinstance(hotspot, np.ndarray) else hotspot)
        sv = _style(style)
        head = np.zeros((self.npix, 4))
        feat = np.zeros((self.npix, 9))
        target = np.zeros((self.npix, 4))
        has = np.zeros(self.npix, np.uint8)
        rc = _load().orc_frame_tail(self._h, _ptr(hv), _ptr(sv), int(K), float(w0), float(w1), _ptr(head),
                                    _ptr(feat), _ptr(target), _ptr(has))
        if rc != 0:
            raise OracleError(f"orc_frame_tail failed: {rc}")
        return head, feat, target, has.astype(bool)

    def approx(self, hotspot, style, method, param=4, w0=0.0, w1=1.0, beta=MBOIT_BETA, eta=MBOIT_ETA):
        """Approximate order-independent resolve per sample pixel (definitions in
        hexfc_oracle.c): method "mlab" (param = k layers) or "mboit" (four power
        moments).  Returns rgba [npix, 4] over the background."""
        hv = np.ascontiguousarray(hotspot_vector(hotspot) if not isinstance(hotspot, np.ndarray) else hotspot)
        sv = _style(style)
        rgba = np.zeros((self.npix, 4))
        m = {"mlab": 1, "mboit": 2}[method]
        rc = _load().orc_frame_approx(self._h, _ptr(hv), _ptr(sv), m, int(param), float(beta), float(eta),
                                      float(w0), float(w1), _ptr(rgba))
        if rc != 0:
            raise OracleError(f"orc_frame_approx failed: {rc}")
        return rgba

    def __del__(self):
        if getattr(self, "_h", None):
            _load().orc_frame_free(self._h)
            self._h = None


def view_depth_range(mesh_pos_q, view_proj):
    """[w0, w1]: range of the clip w of the 8 corners of the bbox of the
    (dequantised) vertex positions, computed with the float camera matrix."""
    P = np.asarray(mesh_pos_q, dtype=np.float64) / 65536.0
    lo, hi = P.min(axis=0), P.max(axis=0)
    M = np.asarray(view_proj, dtype=np.float32).astype(np.float64).reshape(4, 4)
    ws = []
    for c in range(8):
        x = np.array([hi[0] if c & 1 else lo[0], hi[1] if c & 2 else lo[1], hi[2] if c & 4 else lo[2], 1.0])
        ws.append(float(M[3] @ x))
    return min(ws), max(ws)


def render(mesh_synth, cam, hot, style, pixels=None):
    """Convenience: full oracle pass for one view.  Returns a dict."""
    om = Mesh.from_synth(mesh_synth)
    fr = Frame.from_camera(om, cam, pixels)
    count, off, rec = fr.lists()
    rgba, ncand, cand_off, cand = fr.shade(hot, style)
    return dict(mesh=om, frame=fr, count=count, off=off, rec=rec, rgba=rgba, ncand=ncand,
                cand_off=cand_off, cand=cand)
