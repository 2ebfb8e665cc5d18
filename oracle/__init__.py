"""TEST INFRASTRUCTURE ONLY: the CPU oracle for LDNI sampling.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does; it
shares no code with the HIP path.

``sample`` wraps the plain C oracle (``ldni_oracle.c``) that evaluates the
sampling definition of the paper (Sec. 2, Definitions 1-3; accurate face
normals, Sec. 3) ray by ray and triangle by triangle.  ``exact`` holds a
rational-arithmetic micro-oracle for tiny meshes.  The fixed readings of the
paper (pixel-centre formula, tie rule, canonical depth, order) are listed in
``ldni_oracle.h``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldni_oracle.c")
_SRC_BOOL = os.path.join(_HERE, "boolean_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libldni_oracle.so")
_lib = None

AXES = "xyz"


def build(force: bool = True) -> str:
    """Compile the C oracle with IEEE double semantics (no FMA contraction,
    no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-Wall", "-o", tmp, _SRC, _SRC_BOOL, "-lpthread", "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Axis(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("n", ctypes.c_uint64),
                ("offsets", ctypes.POINTER(ctypes.c_uint32)),
                ("depth", ctypes.POINTER(ctypes.c_float)),
                ("normal", ctypes.POINTER(ctypes.c_float)),
                ("tri", ctypes.POINTER(ctypes.c_int32))]


class _Axis64(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("n", ctypes.c_uint64),
                ("offsets", ctypes.POINTER(ctypes.c_uint32)),
                ("depth", ctypes.POINTER(ctypes.c_double)),
                ("normal", ctypes.POINTER(ctypes.c_double)),
                ("tri", ctypes.POINTER(ctypes.c_int32))]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(_SRC),
                                                                          os.path.getmtime(_SRC_BOOL)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_sample_axis.argtypes = [vp, i64, vp, i64, vp, i32, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, i32, i32, i32, i32, ctypes.POINTER(_Axis)]
    lib.oracle_sample_axis.restype = ctypes.c_int
    lib.oracle_axis_free.argtypes = [ctypes.POINTER(_Axis)]
    lib.oracle_sample_axis_f64.argtypes = [vp, i64, vp, i64, vp, i32, ctypes.c_int,
                                           i32, i32, i32, i32, ctypes.POINTER(_Axis64)]
    lib.oracle_sample_axis_f64.restype = ctypes.c_int
    lib.oracle_axis64_free.argtypes = [ctypes.POINTER(_Axis64)]
    lib.oracle_backward_axis.argtypes = [vp, i64, vp, i64, vp, i32, ctypes.c_int,
                                         vp, vp, ctypes.c_uint64, vp, vp, vp]
    lib.oracle_backward_axis.restype = ctypes.c_int
    lib.oracle_pixel_centres.argtypes = [vp, i32, ctypes.c_int, vp, vp]
    lib.oracle_pixel_centres.restype = ctypes.c_int
    pu32, pf32, pi32 = (ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_float),
                        ctypes.POINTER(ctypes.c_int32))
    lib.oracle_boolean.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_double,
                                   ctypes.POINTER(pu32), ctypes.POINTER(pf32), ctypes.POINTER(pf32),
                                   ctypes.POINTER(pi32), ctypes.POINTER(ctypes.c_uint64)]
    lib.oracle_boolean.restype = ctypes.c_int
    lib.oracle_boolean_free.argtypes = [pu32, pf32, pf32, pi32]
    lib.oracle_boolean_free.restype = None
    _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, code):
        names = {1: "invalid argument", 2: "triangle index out of range", 3: "out of memory",
                 4: "sample count overflows u32", 6: "non-finite vertex"}
        super().__init__(f"oracle error {code}: {names.get(code, '?')}")
        self.code = code


@dataclass
class AxisLDNI:
    """One axis of an LDNI in the compact layout: ``offsets[w*w+1]`` and the
    samples of pixel p = j*w + i at ``[offsets[p], offsets[p+1])``."""
    w: int
    offsets: np.ndarray   # uint32 [w*w+1]
    depth: np.ndarray     # float32 [n] (float64 in the f64 variant)
    normal: np.ndarray    # float32 [n,3]
    tri: np.ndarray       # int32 [n]

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    @property
    def counts(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64))


def bbox_f32(bbox) -> np.ndarray:
    """The library takes the box as float32; the oracle sees the same values."""
    return np.asarray(bbox, dtype=np.float32).astype(np.float64)


def _axes(axes):
    if isinstance(axes, str):
        return [AXES.index(c) for c in axes]
    return list(axes)


def _prep(verts, tris):
    v = np.ascontiguousarray(verts, dtype=np.float32).reshape(-1, 3)
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    return v, t


def sample(verts, tris, bbox, w, axes="xyz", brute=False, nthreads=0, window=None):
    """Oracle LDNI sampling; returns ``{axis_index: AxisLDNI}``.

    ``window=(i0, i1, j0, j1)`` restricts sampling to those pixels (the others
    get no samples)."""
    lib = _load()
    v, t = _prep(verts, tris)
    bb = np.ascontiguousarray(bbox_f32(bbox))
    i0, i1, j0, j1 = window if window is not None else (0, w, 0, w)
    out = {}
    for a in _axes(axes):
        ax = _Axis()
        rc = lib.oracle_sample_axis(v.ctypes.data, len(v), t.ctypes.data, len(t), bb.ctypes.data,
                                    int(w), a, int(bool(brute)), int(nthreads),
                                    i0, i1, j0, j1, ctypes.byref(ax))
        if rc != 0:
            lib.oracle_axis_free(ctypes.byref(ax))
            raise OracleError(rc)
        n = int(ax.n)
        npix = int(w) * int(w)
        res = AxisLDNI(
            int(w),
            np.ctypeslib.as_array(ax.offsets, (npix + 1,)).copy(),
            np.ctypeslib.as_array(ax.depth, (max(n, 1),))[:n].copy(),
            np.ctypeslib.as_array(ax.normal, (max(n, 1) * 3,))[:3 * n].reshape(n, 3).copy(),
            np.ctypeslib.as_array(ax.tri, (max(n, 1),))[:n].copy())
        lib.oracle_axis_free(ctypes.byref(ax))
        out[a] = res
    return out


def sample_f64(verts64, tris, bbox, w, axis, window=None) -> AxisLDNI:
    """The same definition evaluated entirely in float64 (pixel centres,
    translation, edge functions, depth, normal), for finite differences."""
    lib = _load()
    v = np.ascontiguousarray(verts64, dtype=np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    bb = np.ascontiguousarray(bbox_f32(bbox))
    i0, i1, j0, j1 = window if window is not None else (0, w, 0, w)
    ax = _Axis64()
    rc = lib.oracle_sample_axis_f64(v.ctypes.data, len(v), t.ctypes.data, len(t), bb.ctypes.data,
                                    int(w), int(axis), i0, i1, j0, j1, ctypes.byref(ax))
    if rc != 0:
        lib.oracle_axis64_free(ctypes.byref(ax))
        raise OracleError(rc)
    n = int(ax.n)
    npix = int(w) * int(w)
    res = AxisLDNI(
        int(w),
        np.ctypeslib.as_array(ax.offsets, (npix + 1,)).copy(),
        np.ctypeslib.as_array(ax.depth, (max(n, 1),))[:n].copy(),
        np.ctypeslib.as_array(ax.normal, (max(n, 1) * 3,))[:3 * n].reshape(n, 3).copy(),
        np.ctypeslib.as_array(ax.tri, (max(n, 1),))[:n].copy())
    lib.oracle_axis64_free(ctypes.byref(ax))
    return res


def backward(verts, tris, bbox, w, axis, ldni: AxisLDNI, grad_depth=None, grad_normal=None):
    """Analytic float64 gradient of sum(gd*depth) + sum(gn.normal) over one
    axis' samples with respect to the vertices; returns float64 [V,3]."""
    lib = _load()
    v, t = _prep(verts, tris)
    bb = np.ascontiguousarray(bbox_f32(bbox))
    off = np.ascontiguousarray(ldni.offsets, dtype=np.uint32)
    tri = np.ascontiguousarray(ldni.tri, dtype=np.int32)
    gd = None if grad_depth is None else np.ascontiguousarray(grad_depth, dtype=np.float32)
    gn = None if grad_normal is None else np.ascontiguousarray(grad_normal, dtype=np.float32)
    grad = np.zeros((len(v), 3), dtype=np.float64)
    rc = lib.oracle_backward_axis(v.ctypes.data, len(v), t.ctypes.data, len(t), bb.ctypes.data,
                                  int(w), int(axis), off.ctypes.data, tri.ctypes.data,
                                  int(ldni.n), None if gd is None else gd.ctypes.data,
                                  None if gn is None else gn.ctypes.data, grad.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return grad


def pixel_centres(bbox, w, axis):
    lib = _load()
    bb = np.ascontiguousarray(bbox_f32(bbox))
    cu = np.zeros(w, np.float32)
    cv = np.zeros(w, np.float32)
    rc = lib.oracle_pixel_centres(bb.ctypes.data, int(w), int(axis), cu.ctypes.data, cv.ctypes.data)
    if rc != 0:
        raise OracleError(rc)
    return cu, cv
