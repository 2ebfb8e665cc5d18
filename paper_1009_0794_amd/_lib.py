"""ctypes declarations of the C ABI in ``include/ldni.h`` (argument
marshalling only; every step of sampling runs in the HIP library)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LDNI_LIBRARY", os.path.join(HERE, "libldni.so"))

c_u32p = ctypes.POINTER(ctypes.c_uint32)
c_f32p = ctypes.POINTER(ctypes.c_float)
c_i32p = ctypes.POINTER(ctypes.c_int32)


class AxisView(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("max_layers", ctypes.c_uint32),
                ("n_samples", ctypes.c_uint64), ("offsets", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("tri", ctypes.c_void_p), ("normal_rgb8", ctypes.c_void_p)]


class MeshDesc(ctypes.Structure):
    _fields_ = [("verts", ctypes.c_void_p), ("n_verts", ctypes.c_int64),
                ("tris", ctypes.c_void_p), ("n_tris", ctypes.c_int64),
                ("bbox", ctypes.c_float * 6), ("w", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double)]


STATUS = {0: "LDNI_OK", 1: "LDNI_ERR_INVALID_ARG", 2: "LDNI_ERR_INDEX",
          3: "LDNI_ERR_OUT_OF_MEMORY", 4: "LDNI_ERR_OVERFLOW", 5: "LDNI_ERR_DEVICE",
          6: "LDNI_ERR_NONFINITE"}


class LDNIError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"{STATUS.get(code, code)}: {detail}")
        self.code = code
        self.detail = detail


_lib = None


def lib():
    """The loaded ``libldni.so``; raises if it has not been built (there is no
    fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    st = ctypes.c_int
    L.ldni_sample.argtypes = [vp, i64, vp, i64, vp, i32, u32, vp, ctypes.POINTER(vp)]
    L.ldni_sample.restype = st
    L.ldni_result_axis.argtypes = [vp, ctypes.c_int, ctypes.POINTER(AxisView)]
    L.ldni_result_axis.restype = st
    L.ldni_free.argtypes = [vp]
    L.ldni_free.restype = None
    L.ldni_trim.argtypes = []
    L.ldni_trim.restype = st
    L.ldni_sample_begin.argtypes = [vp, i64, vp, i64, vp, i32, u32, ctypes.POINTER(vp), vp,
                                    ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_uint64)]
    L.ldni_sample_begin.restype = st
    L.ldni_sample_finish.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.ldni_sample_finish.restype = st
    L.ldni_sample_finish_rgb8.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.ldni_sample_finish_rgb8.restype = st
    L.ldni_plan_free.argtypes = [vp]
    L.ldni_plan_free.restype = None
    L.ldni_plan_max_layers.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32)]
    L.ldni_plan_max_layers.restype = st
    L.ldni_status_string.argtypes = [st]
    L.ldni_status_string.restype = ctypes.c_char_p
    L.ldni_last_error.argtypes = []
    L.ldni_last_error.restype = ctypes.c_char_p
    L.ldni_set_tile_shape.argtypes = [i32, i32]
    L.ldni_set_tile_shape.restype = st
    L.ldni_backward.argtypes = [vp, i64, vp, i64, vp, i32, u32, ctypes.POINTER(AxisView),
                                ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp]
    L.ldni_backward.restype = st
    L.ldni_backward_noalloc.argtypes = [vp, i64, vp, i64, vp, i32, u32, ctypes.POINTER(AxisView),
                                ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp]
    L.ldni_backward_noalloc.restype = st
    L.ldni_batch_create.argtypes = [i32, ctypes.POINTER(MeshDesc), u32, vp, ctypes.POINTER(vp)]
    L.ldni_batch_create.restype = st
    L.ldni_sample_batch.argtypes = [i32, ctypes.POINTER(MeshDesc), u32, vp, ctypes.POINTER(vp)]
    L.ldni_sample_batch.restype = st
    L.ldni_batch_run.argtypes = [vp, vp]
    L.ldni_batch_run.restype = st
    L.ldni_batch_axis.argtypes = [vp, i32, ctypes.c_int, ctypes.POINTER(AxisView)]
    L.ldni_batch_axis.restype = st
    L.ldni_batch_free.argtypes = [vp]
    L.ldni_batch_free.restype = None
    L.ldni_boolean.argtypes = [ctypes.POINTER(AxisView), ctypes.POINTER(AxisView), i32, ctypes.c_float, i32,
                               vp, ctypes.POINTER(vp)]
    L.ldni_boolean.restype = st
    L.ldni_classify_nodes.argtypes = [ctypes.POINTER(AxisView), ctypes.POINTER(ctypes.c_float), vp,
                                      ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), vp]
    L.ldni_classify_nodes.restype = st
    L.ldni_node_words.argtypes = [i32, ctypes.POINTER(ctypes.c_uint64)]
    L.ldni_node_words.restype = st
    L.ldni_offset.argtypes = [ctypes.POINTER(AxisView), ctypes.POINTER(ctypes.c_float), ctypes.c_float,
                              ctypes.c_float, vp, ctypes.POINTER(vp)]
    L.ldni_offset.restype = st
    L.ldni_profile_enable.argtypes = [ctypes.c_int]
    L.ldni_profile_enable.restype = st
    L.ldni_profile_read.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
    L.ldni_profile_read.restype = st
    _lib = L
    return L


def check(code: int) -> None:
    if code != 0:
        detail = lib().ldni_last_error().decode(errors="replace")
        raise LDNIError(int(code), detail)


_hip = None


def hip():
    """The HIP runtime (for device-to-device copies of library-owned views)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int, ctypes.c_void_p]
        _hip.hipMemcpyAsync.restype = ctypes.c_int
    return _hip


def exported_symbols():
    """Names of the C ABI functions declared in include/ldni.h."""
    return ["ldni_sample", "ldni_result_axis", "ldni_free", "ldni_trim", "ldni_sample_begin",
            "ldni_sample_finish", "ldni_plan_free", "ldni_plan_max_layers",
            "ldni_status_string", "ldni_last_error", "ldni_set_tile_shape",
            "ldni_profile_enable", "ldni_profile_read", "ldni_backward", "ldni_batch_create",
            "ldni_batch_run", "ldni_batch_axis", "ldni_batch_free", "ldni_sample_batch",
            "ldni_boolean", "ldni_sample_finish_rgb8", "ldni_classify_nodes", "ldni_node_words",
            "ldni_offset", "ldni_backward_noalloc"]
