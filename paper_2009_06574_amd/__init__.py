"""hexfc: MI355X-native focus+context hex-mesh renderer (Python binding).

Thin ctypes binding of ``libhexfc.so`` (include/hexfc.h).  It only marshals
arguments: every step of the render path runs in the library's HIP kernels.
PyTorch provides device memory (workspace, outputs) and the current stream.
There is no CPU fallback: if the library has not been built, ``load()``
raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhexfc.so")

STATUS = {0: "HEXFC_OK", -1: "HEXFC_EINVAL", -2: "HEXFC_ERANGE", -3: "HEXFC_ENOMEM",
          -4: "HEXFC_EOVERFLOW", -5: "HEXFC_EDEVICE", -6: "HEXFC_ESTATE"}

# every entry point declared in include/hexfc.h
ABI_SYMBOLS = (
    "hexfc_create", "hexfc_destroy", "hexfc_set_workspace", "hexfc_upload_mesh",
    "hexfc_build_fragment_lists", "hexfc_resolve", "hexfc_render_frame", "hexfc_set_tuning",
    "hexfc_get_frame_stats", "hexfc_get_total_fragments", "hexfc_export_sorted_lists",
    "hexfc_set_profiling", "hexfc_get_kernel_times", "hexfc_render_batch", "hexfc_batch_status",
    "hexfc_autotune", "hexfc_resolve_approx", "hexfc_resolve_learned", "hexfc_resolve_learned_noalloc", "hexfc_learned_features",
    "hexfc_mlp_param_count",
    "hexfc_mlp_forward", "hexfc_mlp_loss", "hexfc_mlp_backward", "hexfc_mlp_adam_step",
    "hexfc_build_lod", "hexfc_status_string", "hexfc_last_error",
)


class HexfcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class CCamera(ct.Structure):
    _fields_ = [("view_proj", ct.c_float * 16), ("width", ct.c_int32), ("height", ct.c_int32)]


class CHotspot(ct.Structure):
    _fields_ = [("center", ct.c_float * 3), ("radius", ct.c_float)]


class CStyle(ct.Structure):
    _fields_ = [("w_base", ct.c_float), ("k_focus", ct.c_float), ("halo_width", ct.c_float),
                ("halo_alpha", ct.c_float), ("darken", ct.c_float), ("accent_s", ct.c_float),
                ("accent_brighten", ct.c_float), ("delta", ct.c_float), ("lod", ct.c_int32),
                ("tf_rgb_lo", ct.c_float * 3), ("tf_rgb_hi", ct.c_float * 3),
                ("tf_a_lo", ct.c_float), ("tf_a_hi", ct.c_float), ("bg", ct.c_float * 3),
                ("lens_mode", ct.c_int32), ("desaturate", ct.c_float),
                ("sil_alpha", ct.c_float), ("sil_tau", ct.c_float)]


_lib = None


class CLodInfo(ct.Structure):
    _fields_ = [("sheets", ct.c_int64), ("edges", ct.c_int64), ("faces", ct.c_int64),
                ("singular_edges", ct.c_int64), ("merges", ct.c_int64 * 3), ("levels", ct.c_int32),
                ("components_left", ct.c_int32)]


def load():
    """Load libhexfc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2009_06574_amd.build.build()")
    lib = ct.CDLL(LIB_PATH)
    P, i64, st = ct.c_void_p, ct.c_int64, ct.c_int
    sig = {
        "hexfc_create": ([ct.c_int, ct.POINTER(P)], st),
        "hexfc_destroy": ([P], None),
        "hexfc_set_workspace": ([P, P, ct.c_size_t], st),
        "hexfc_upload_mesh": ([P, P, i64, P, i64, P, P], st),
        "hexfc_build_fragment_lists": ([P, ct.POINTER(CCamera), P, P], st),
        "hexfc_resolve": ([P, ct.POINTER(CHotspot), ct.POINTER(CStyle), P, P], st),
        "hexfc_render_frame": ([P, ct.POINTER(CCamera), ct.POINTER(CHotspot), ct.POINTER(CStyle), P, P], st),
        "hexfc_set_tuning": ([P, ct.c_int, ct.c_int, ct.c_int], st),
        "hexfc_get_frame_stats": ([P, P, ct.c_int], st),
        "hexfc_get_total_fragments": ([P, P], st),
        "hexfc_export_sorted_lists": ([P, P, P, P, P], st),
        "hexfc_set_profiling": ([P, ct.c_int], st),
        "hexfc_get_kernel_times": ([P, P, P, ct.c_int], st),
        "hexfc_render_batch": ([P, ct.c_int, P, P, P, P, P], st),
        "hexfc_batch_status": ([P, P, P, P], st),
        "hexfc_autotune": ([P, ct.c_int, P, P, P, P, ct.c_char_p, P, P], st),
        "hexfc_resolve_approx": ([P, ct.POINTER(CHotspot), ct.POINTER(CStyle), ct.c_int, ct.c_int, P, P], st),
        "hexfc_resolve_learned": ([P, ct.POINTER(CHotspot), ct.POINTER(CStyle), P, ct.c_int, ct.c_float, P, P, P],
                                  st),
        "hexfc_resolve_learned_noalloc": ([P, ct.POINTER(CHotspot), ct.POINTER(CStyle), P, ct.c_int, ct.c_float, P,
                                           P, P], st),
        "hexfc_learned_features": ([P, ct.POINTER(CHotspot), ct.POINTER(CStyle), ct.c_int, P, P, P, P, i64, P, P],
                                   st),
        "hexfc_mlp_param_count": ([], i64),
        "hexfc_mlp_forward": ([P, P, i64, P, P], st),
        "hexfc_mlp_loss": ([P, P, i64, ct.c_float, P, P, P], st),
        "hexfc_mlp_backward": ([P, P, P, i64, P, P], st),
        "hexfc_mlp_adam_step": ([P, P, P, P, ct.c_float, ct.c_float, ct.c_float, ct.c_float, ct.c_int, P], st),
        "hexfc_build_lod": ([P, i64, i64, ct.c_int32, P, ct.POINTER(CLodInfo)], st),
        "hexfc_status_string": ([st], ct.c_char_p),
        "hexfc_last_error": ([P], ct.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def camera_struct(cam) -> CCamera:
    c = CCamera()
    vp = np.asarray(cam.view_proj, dtype=np.float32).reshape(16)
    c.view_proj[:] = [float(x) for x in vp]
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def hotspot_struct(h) -> CHotspot:
    c = CHotspot()
    c.center[:] = [float(x) for x in h.center]
    c.radius = float(h.radius)
    return c


def style_struct(s) -> CStyle:
    c = CStyle()
    for k in ("w_base", "k_focus", "halo_width", "halo_alpha", "darken", "accent_s", "accent_brighten", "delta"):
        setattr(c, k, float(getattr(s, k)))
    c.lod = int(s.lod)
    c.tf_rgb_lo[:] = [float(x) for x in s.tf_rgb_lo]
    c.tf_rgb_hi[:] = [float(x) for x in s.tf_rgb_hi]
    c.tf_a_lo, c.tf_a_hi = float(s.tf_a_lo), float(s.tf_a_hi)
    c.bg[:] = [float(x) for x in s.bg]
    c.lens_mode = int(getattr(s, "lens_mode", 0))
    c.desaturate = float(getattr(s, "desaturate", 0.0))
    c.sil_alpha = float(getattr(s, "sil_alpha", 0.0))
    c.sil_tau = float(getattr(s, "sil_tau", 0.02))
    return c


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


class Renderer:
    """One hexfc context on one GPU."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = torch.device("cuda", device)
        h = ct.c_void_p()
        self._check(self.lib.hexfc_create(device, ct.byref(h)), None)
        self.ctx = h
        self.workspace = None
        self.W = self.H = 0

    def _check(self, status, ctx="self"):
        if status != 0:
            msg = ""
            if ctx is not None and getattr(self, "ctx", None):
                msg = (self.lib.hexfc_last_error(self.ctx) or b"").decode()
            raise HexfcError(status, msg)

    def _stream(self):
        return ct.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hexfc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ setup
    def set_workspace(self, nbytes: int):
        nbytes = int(nbytes)
        self.workspace = self.torch.empty(max(nbytes, 256), dtype=self.torch.uint8, device=self.device)
        self._check(self.lib.hexfc_set_workspace(self.ctx, _ptr(self.workspace), nbytes))

    def set_tuning(self, tile_w: int = 8, tile_h: int = 8, t_sort: int = 16):
        self._check(self.lib.hexfc_set_tuning(self.ctx, int(tile_w), int(tile_h), int(t_sort)))

    def upload_mesh(self, xyz, hexes, cell_scalar=None, cell_edge_level=None):
        xyz = np.ascontiguousarray(xyz, dtype=np.float32)
        hexes = np.ascontiguousarray(hexes, dtype=np.int32)
        sc = None if cell_scalar is None else np.ascontiguousarray(cell_scalar, dtype=np.float32)
        lv = None if cell_edge_level is None else np.ascontiguousarray(cell_edge_level, dtype=np.uint8)
        p = lambda a: None if a is None else a.ctypes.data_as(ct.c_void_p)
        self._check(self.lib.hexfc_upload_mesh(self.ctx, p(xyz), xyz.shape[0], p(hexes), hexes.shape[0],
                                               p(sc), p(lv)))

    def upload(self, mesh):
        """Upload an object with xyz / hex / cell_scalar / cell_edge_level attributes."""
        self.upload_mesh(mesh.xyz, mesh.hex, getattr(mesh, "cell_scalar", None),
                         getattr(mesh, "cell_edge_level", None))

    # ------------------------------------------------------------ frames
    def build(self, cam, want_counts: bool = False):
        c = camera_struct(cam)
        counts = None
        if want_counts:
            counts = self.torch.empty((c.height, c.width), dtype=self.torch.int32, device=self.device)
        self._check(self.lib.hexfc_build_fragment_lists(self.ctx, ct.byref(c), _ptr(counts), self._stream()))
        self.W, self.H = c.width, c.height
        return counts

    def resolve(self, hot, style, out=None):
        if out is None:
            out = self.torch.empty((self.H, self.W, 4), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.hexfc_resolve(self.ctx, ct.byref(hotspot_struct(hot)), ct.byref(style_struct(style)),
                                           _ptr(out), self._stream()))
        return out

    def render(self, cam, hot, style, out=None):
        c = camera_struct(cam)
        if out is None:
            out = self.torch.empty((c.height, c.width, 4), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.hexfc_render_frame(self.ctx, ct.byref(c), ct.byref(hotspot_struct(hot)),
                                                ct.byref(style_struct(style)), _ptr(out), self._stream()))
        self.W, self.H = c.width, c.height
        return out

    def render_batch(self, cams, hots, styles, out=None):
        """n views of one viewport in one captured graph; returns [n, H, W, 4]."""
        n = len(cams)
        cc = (CCamera * n)(*[camera_struct(c) for c in cams])
        hh = (CHotspot * n)(*[hotspot_struct(h) for h in hots])
        ss = (CStyle * n)(*[style_struct(s) for s in styles])
        W, H = cc[0].width, cc[0].height
        if out is None:
            out = self.torch.empty((n, H, W, 4), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.hexfc_render_batch(self.ctx, n, ct.cast(cc, ct.c_void_p), ct.cast(hh, ct.c_void_p),
                                                ct.cast(ss, ct.c_void_p), _ptr(out), self._stream()))
        self.W, self.H = W, H
        return out

    def batch_status(self):
        """(fragments, overflowed) of the last batch; waits for the stream."""
        f = ct.c_uint64()
        o = ct.c_int()
        self._check(self.lib.hexfc_batch_status(self.ctx, ct.byref(f), ct.byref(o), self._stream()))
        return int(f.value), bool(o.value)

    def autotune(self, cams, hots, styles, cache_path=None, out=None):
        """Choose tile shape and sort switch by timing; returns (tile_w, tile_h, t_sort)."""
        n = len(cams)
        cc = (CCamera * n)(*[camera_struct(c) for c in cams])
        hh = (CHotspot * n)(*[hotspot_struct(h) for h in hots])
        ss = (CStyle * n)(*[style_struct(s) for s in styles])
        if out is None:
            out = self.torch.empty((n, cc[0].height, cc[0].width, 4), dtype=self.torch.float32, device=self.device)
        choice = (ct.c_int * 3)()
        path = None if cache_path is None else str(cache_path).encode()
        self._check(self.lib.hexfc_autotune(self.ctx, n, ct.cast(cc, ct.c_void_p), ct.cast(hh, ct.c_void_p),
                                            ct.cast(ss, ct.c_void_p), _ptr(out), path, ct.cast(choice, ct.c_void_p),
                                            self._stream()))
        return tuple(int(x) for x in choice)

    def export_sorted_lists(self):
        """(counts int32 [H*W], off int64 [H*W+1], rec int64 [F]) in row-major pixel order;
        uint32/uint64 bit patterns stored in signed tensors."""
        n = self.W * self.H
        F = self.total_fragments()
        t = self.torch
        counts = t.empty(n, dtype=t.int32, device=self.device)
        off = t.empty(n + 1, dtype=t.int64, device=self.device)
        rec = t.empty(max(F, 1), dtype=t.int64, device=self.device)
        self._check(self.lib.hexfc_export_sorted_lists(self.ctx, _ptr(counts), _ptr(off), _ptr(rec), self._stream()))
        return counts, off, rec[:F]

    def total_fragments(self) -> int:
        v = ct.c_uint64()
        self._check(self.lib.hexfc_get_total_fragments(self.ctx, ct.byref(v)))
        return int(v.value)

    def frame_stats(self) -> dict:
        """Statistics of the last frame (waits for it)."""
        a = (ct.c_uint64 * 32)()
        self._check(self.lib.hexfc_get_frame_stats(self.ctx, a, 32))
        return dict(bins=int(a[0]), fragments=int(a[1]), passes=int(a[2]), flags=int(a[4]),
                    classes=[int(a[8 + i]) for i in range(8)],
                    class_fragments=[int(a[16 + i]) for i in range(8)],
                    fallback=[int(a[24 + i]) for i in range(8)])

    KERNELS = ("transform", "bin_count", "bin_scatter", "count", "scan", "classify", "plan", "fill", "resolve",
               "tail_features", "mlp_apply", "fallback") + tuple(f"resolve_c{c}" for c in range(8))

    APPROX_METHODS = {"mlab": 1, "moments": 2}

    def resolve_approx(self, hot, style, method="mlab", k=4, out=None):
        """Approximate order-independent resolve of the last built lists:
        "mlab" (k blending layers) or "moments" (four power moments)."""
        if out is None:
            out = self.torch.empty((self.H, self.W, 4), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.hexfc_resolve_approx(self.ctx, ct.byref(hotspot_struct(hot)),
                                                  ct.byref(style_struct(style)), self.APPROX_METHODS[method],
                                                  int(k), _ptr(out), self._stream()))
        return out

    # ------------------------------------------------------------ learned tail
    def learned_features(self, hot, style, K: int = 8, with_target: bool = False) -> dict:
        """Rows of the learned resolve for the last built lists: head [r,4], feat [r,9],
        target [r,4] (exact tail, if asked) and pix [r] (y*W+x, int32)."""
        rows = ct.c_int64()
        hs, ss = hotspot_struct(hot), style_struct(style)
        self._check(self.lib.hexfc_learned_features(self.ctx, ct.byref(hs), ct.byref(ss), int(K), None, None, None,
                                                    None, 0, ct.byref(rows), self._stream()))
        r = int(rows.value)
        t = self.torch
        out = dict(head=t.empty((max(r, 1), 4), dtype=t.float32, device=self.device),
                   feat=t.empty((max(r, 1), 9), dtype=t.float32, device=self.device),
                   target=t.empty((max(r, 1), 4), dtype=t.float32, device=self.device) if with_target else None,
                   pix=t.empty(max(r, 1), dtype=t.int32, device=self.device))
        self._check(self.lib.hexfc_learned_features(self.ctx, ct.byref(hs), ct.byref(ss), int(K), _ptr(out["head"]),
                                                    _ptr(out["feat"]), _ptr(out["target"]), _ptr(out["pix"]),
                                                    max(r, 1), ct.byref(rows), self._stream()))
        return {k: (None if v is None else v[:r]) for k, v in out.items()}

    def resolve_learned(self, hot, style, params, K: int = 8, conf_min: float = 0.5, out=None, mask=True,
                        noalloc: bool = False):
        """Learned-tail resolve of the last built lists: (rgba [H,W,4], mask [H,W] uint8 or None).
        noalloc: the allocation-free entry point (static per-GPU staging; the
        caller's buffers are still allocated here when not given)."""
        t = self.torch
        if out is None:
            out = t.empty((self.H, self.W, 4), dtype=t.float32, device=self.device)
        m = None
        if mask is True:
            m = t.empty((self.H, self.W), dtype=t.uint8, device=self.device)
        elif mask is not None and mask is not False:
            m = mask
        params = _f32(params, self.device)
        fn = self.lib.hexfc_resolve_learned_noalloc if noalloc else self.lib.hexfc_resolve_learned
        self._check(fn(self.ctx, ct.byref(hotspot_struct(hot)), ct.byref(style_struct(style)), _ptr(params), int(K),
                       float(conf_min), _ptr(out), _ptr(m), self._stream()))
        return out, m


    def set_profiling(self, on: bool = True):
        self._check(self.lib.hexfc_set_profiling(self.ctx, 1 if on else 0))

    def kernel_times(self) -> dict:
        """Accumulated (ms, launches) per kernel since the last call (waits for the events)."""
        k = len(self.KERNELS)
        ms = (ct.c_double * k)()
        n = (ct.c_uint64 * k)()
        self._check(self.lib.hexfc_get_kernel_times(self.ctx, ms, n, k))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNELS) if n[i]}


# ---------------------------------------------------------------- learned-tail network kernels
def _f32(t, device=None):
    import torch
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float32))
    if device is not None and t.device != torch.device(device):
        t = t.to(device)
    if t.dtype != torch.float32 or not t.is_contiguous():
        t = t.to(torch.float32).contiguous()
    if t.device.type != "cuda":
        raise ValueError("learned-tail kernels need CUDA (HIP) tensors")
    return t


def _status(rc):
    if rc != 0:
        raise HexfcError(rc, "learned-tail kernel call failed")


def _cur_stream(t):
    import torch
    return ct.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def mlp_param_count() -> int:
    return int(load().hexfc_mlp_param_count())


def mlp_forward(params, x, y=None):
    """y [n,5] = MLP(x [n,9]) on the GPU."""
    import torch
    lib = load()
    x = _f32(x)
    params = _f32(params, x.device)
    n = x.shape[0]
    if y is None:
        y = torch.empty((n, 5), dtype=torch.float32, device=x.device)
    _status(lib.hexfc_mlp_forward(_ptr(params), _ptr(x), n, _ptr(y), _cur_stream(x)))
    return y


def mlp_loss(y, target, dy=None, loss_sum=None, conf_tol=2e-3):
    """(dy [n,5], loss_sum [1]): loss_sum accumulates the per-row losses; the
    confidence label is max_c |y_c - t_c| < conf_tol."""
    import torch
    lib = load()
    y, target = _f32(y), _f32(target)
    n = y.shape[0]
    if dy is None:
        dy = torch.empty((n, 5), dtype=torch.float32, device=y.device)
    if loss_sum is None:
        loss_sum = torch.zeros(1, dtype=torch.float32, device=y.device)
    _status(lib.hexfc_mlp_loss(_ptr(y), _ptr(target), n, float(conf_tol), _ptr(dy), _ptr(loss_sum),
                               _cur_stream(y)))
    return dy, loss_sum


def mlp_backward(params, x, dy, grad=None):
    """grad += d(sum dy*y)/d params (a zeroed gradient is allocated if none is given)."""
    import torch
    lib = load()
    x, dy = _f32(x), _f32(dy)
    params = _f32(params, x.device)
    if grad is None:
        grad = torch.zeros(mlp_param_count(), dtype=torch.float32, device=x.device)
    _status(lib.hexfc_mlp_backward(_ptr(params), _ptr(x), _ptr(dy), x.shape[0], _ptr(grad), _cur_stream(x)))
    return grad


def mlp_adam_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float32 CUDA tensors params, m, v."""
    lib = load()
    for t in (params, m, v, grad):
        if t.dtype.__repr__() != "torch.float32" or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError("params, m, v and grad must be contiguous float32 CUDA tensors")
    _status(lib.hexfc_mlp_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), float(lr), float(beta1),
                                    float(beta2), float(eps), int(step), _cur_stream(params)))


def build_lod(hexes, V: int, n_threads: int = 0):
    """Sheet-based LoD levels of a hexahedral mesh (host C++ in the library):
    returns (cell_edge_level uint8 [C, 12], info dict)."""
    lib = load()
    h = np.ascontiguousarray(hexes, dtype=np.int32).reshape(-1, 8)
    out = np.zeros((h.shape[0], 12), dtype=np.uint8)
    info = CLodInfo()
    rc = lib.hexfc_build_lod(h.ctypes.data_as(ct.c_void_p), h.shape[0], int(V), int(n_threads),
                             out.ctypes.data_as(ct.c_void_p), ct.byref(info))
    if rc != 0:
        raise HexfcError(rc, "hexfc_build_lod failed")
    return out, {"sheets": info.sheets, "edges": info.edges, "faces": info.faces,
                 "singular_edges": info.singular_edges, "merges": list(info.merges),
                 "levels": info.levels, "components_left": info.components_left}
