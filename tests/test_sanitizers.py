"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code.

The FP64 oracle (oracle/hexfc_oracle.c) and the library's host-only LoD
builder (csrc/lod.cpp, behind hexfc_build_lod) are compiled again with
-fsanitize=address,undefined (gcc / g++, no recovery: the first report ends
the process) and driven through their whole interface in a child process
with the ASan runtime preloaded: meshes with boundary and jittered cells,
perspective views with the near plane inside the mesh and grazing views,
list building, shading with every style branch, the learned-tail features
and the approximate resolves; sheet-based LoD of grids, box grids, polygon
prisms and relabelled meshes on one and several threads.  The child must
exit cleanly with no sanitizer report, and the sanitized LoD must equal the
oracle's.

The library's HIP host code (context, upload, frame orchestration) is not
covered here: it cannot run without a GPU.
"""
from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.fixture(scope="module")
def san_libs(tmp_path_factory):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's ASan runtime is not installed")
    d = tmp_path_factory.mktemp("san")
    orc = str(d / "liboracle_san.so")
    lod = str(d / "liblod_san.so")
    subprocess.check_call(["gcc", "-std=c11", "-fopenmp", "-fPIC", "-shared", *SAN, "-o", orc,
                           os.path.join(ROOT, "oracle", "hexfc_oracle.c"), "-lm"])
    subprocess.check_call(["g++", "-std=c++17", "-pthread", "-fPIC", "-shared", *SAN,
                           "-I", os.path.join(ROOT, "include"), "-o", lod,
                           os.path.join(ROOT, "paper_2009_06574_amd", "csrc", "lod.cpp")])
    return dict(asan=asan, oracle=orc, lod=lod, dir=str(d))


CHILD = r'''
import ctypes as ct, sys
import numpy as np
sys.path.insert(0, ROOT)
import synth, oracle
from tests.test_lod import relabel

def views(mesh, n, W, H, seed):
    cams, hots, sts = synth.random_views(mesh, n, W, H, seed)
    lo, hi = mesh.bbox()
    c = 0.5 * (lo + hi)
    # eye inside the mesh (near plane cuts it) and a grazing view along a face plane
    cams.append(synth.make_camera(c, c + np.array([1.0, 0.2, 0.1]), W, H))
    cams.append(synth.make_camera((lo[0] - 1.0, lo[1], c[2]), (hi[0], lo[1], c[2]), W, H))
    hots += [hots[0], hots[-1]]
    sts += [synth.default_style(cams[-2]), synth.default_style(cams[-1])]
    return list(zip(cams, hots, sts))

for mesh in (synth.config0()[0], synth.jittered_grid(5, 0.35, seed=3)):
    om = oracle.Mesh.from_synth(mesh)
    om.boundary()
    P = om.export()["pos_q"]
    for cam, hot, st in views(mesh, 2, 48, 40, seed=11):
        fr = oracle.Frame.from_camera(om, cam)
        count, off, rec = fr.lists()
        fr.shade(hot, st)
        fr.shade(hot, synth.default_style(cam, lod=0.0, delta=0.0, accent_s=3.0))
        w0, w1 = oracle.view_depth_range(P, cam.view_proj)
        for K in (1, 4):
            fr.tail(hot, st, K, w0, w1)
        fr.approx(hot, st, "mlab", 4, w0, w1)
        fr.approx(hot, st, "mboit", 0, w0, w1)

lib = ct.CDLL(LOD)
class Info(ct.Structure):
    _fields_ = [("sheets", ct.c_int64), ("edges", ct.c_int64), ("faces", ct.c_int64),
                ("singular_edges", ct.c_int64), ("merges", ct.c_int64 * 3), ("levels", ct.c_int32),
                ("components_left", ct.c_int32)]
out = {}
meshes = [("grid4", synth.grid_cells(4), 125), ("grid5", synth.grid_cells(5), 216)]
b = synth.box_grid(3, 2, 4)
meshes.append(("box", b.hex, b.V))
p = synth.polygon_prism(5, 2, 2)
meshes.append(("prism", p.hex, p.V))
meshes.append(("prism_rel", relabel(p.hex, p.V, 7), p.V))
for name, h, V in meshes:
    h = np.ascontiguousarray(h, dtype=np.int32).reshape(-1, 8)
    for nt in (1, 3):
        lv = np.zeros((h.shape[0], 12), np.uint8)
        info = Info()
        rc = lib.hexfc_build_lod(h.ctypes.data_as(ct.c_void_p), ct.c_int64(h.shape[0]), ct.c_int64(V),
                                 ct.c_int32(nt), lv.ctypes.data_as(ct.c_void_p), ct.byref(info))
        assert rc == 0, (name, rc)
        out[f"{name}_{nt}"] = lv
        out[f"{name}_hex"] = h
np.savez(OUT, **out)
print("child done", flush=True)
'''


def test_host_code_under_asan_and_ubsan(san_libs):
    out = os.path.join(san_libs["dir"], "lod_levels.npz")
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = san_libs["asan"] + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HEXFC_ORACLE_LIB"] = san_libs["oracle"]
    env["OMP_NUM_THREADS"] = "4"
    code = f"ROOT = {ROOT!r}\nLOD = {san_libs['lod']!r}\nOUT = {out!r}\n" + CHILD
    p = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    report = p.stdout[-4000:] + p.stderr[-8000:]
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, report
    assert p.returncode == 0 and "child done" in p.stdout, report
    # the sanitized LoD builder agrees with the oracle
    from oracle import lod
    got = np.load(out)
    for key in got.files:
        if key.endswith("_hex"):
            name = key[:-4]
            want, _ = lod.sheet_lod(got[key])
            for nt in (1, 3):
                assert np.array_equal(got[f"{name}_{nt}"], want), (name, nt)
