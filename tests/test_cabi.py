"""The C ABI library on the host: it loads, exports every function that
include/ldni.h declares, and rejects bad arguments before any GPU call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldni.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ldni_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1009_0794_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "ldni_sample" in names and "ldni_free" in names
    for n in names:
        assert hasattr(L, n), n
    from paper_1009_0794_amd import _lib
    assert sorted(_lib.exported_symbols()) == names


def _call(L, verts=1, nv=3, tris=1, nt=1, bbox=(0, 0, 0, 1, 1, 1), w=8, mask=7):
    bb = (ctypes.c_float * 6)(*bbox) if bbox is not None else None
    out = ctypes.c_void_p(123)
    rc = L.ldni_sample(verts, nv, tris, nt, bb, w, mask, None, ctypes.byref(out))
    return rc, out.value


@pytest.mark.parametrize("kw", [
    dict(w=0), dict(w=16385), dict(w=-3), dict(mask=0), dict(mask=8), dict(mask=256), dict(mask=256 | 8),
    dict(mask=512 | 7),
    dict(bbox=(0, 0, 0, 0, 1, 1)), dict(bbox=(0, 0, 0, 1, -1, 1)),
    dict(bbox=(0, 0, float("nan"), 1, 1, 1)), dict(bbox=(0, 0, 0, float("inf"), 1, 1)),
    dict(nv=-1), dict(nt=-1), dict(verts=None), dict(tris=None), dict(bbox=None),
    dict(nt=2 ** 31),
])
def test_invalid_arguments_rejected_on_host(L, kw):
    rc, out = _call(L, **kw)
    assert rc == 1
    assert out is None
    assert L.ldni_last_error().decode()


def test_status_strings(L):
    for code, name in [(0, "LDNI_OK"), (1, "LDNI_ERR_INVALID_ARG"), (2, "LDNI_ERR_INDEX"),
                       (3, "LDNI_ERR_OUT_OF_MEMORY"), (4, "LDNI_ERR_OVERFLOW"),
                       (5, "LDNI_ERR_DEVICE"), (6, "LDNI_ERR_NONFINITE")]:
        assert L.ldni_status_string(code).decode() == name
    assert L.ldni_status_string(99).decode() == "LDNI_ERR_UNKNOWN"


def test_tile_shape_validation(L):
    assert L.ldni_set_tile_shape(7, 8) == 1
    assert L.ldni_set_tile_shape(64, 32) == 1
    assert L.ldni_set_tile_shape(32, 65) == 1
    assert L.ldni_set_tile_shape(64, 16) == 0
    assert L.ldni_set_tile_shape(0, 4) == 1
    assert L.ldni_set_tile_shape(32, 32) == 0
    assert L.ldni_set_tile_shape(0, 0) == 0


def test_result_axis_rejects_null(L):
    from paper_1009_0794_amd import _lib
    v = _lib.AxisView()
    assert L.ldni_result_axis(None, 0, ctypes.byref(v)) == 1
    L.ldni_free(None)  # NULL-safe
    L.ldni_plan_free(None)


def test_begin_rejects_missing_offsets(L):
    bb = (ctypes.c_float * 6)(0, 0, 0, 1, 1, 1)
    offs = (ctypes.c_void_p * 3)(None, None, None)
    plan = ctypes.c_void_p()
    n = (ctypes.c_uint64 * 3)()
    assert L.ldni_sample_begin(1, 3, 1, 1, bb, 8, 1, offs, None, ctypes.byref(plan), n) == 1
    assert plan.value is None


def test_python_binding_refuses_host_tensors():
    import torch
    import paper_1009_0794_amd as ldni
    with pytest.raises(ValueError):
        ldni.sample(torch.zeros(3, 3), torch.zeros(1, 3, dtype=torch.int32), (0, 0, 0, 1, 1, 1), 8)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_1009_0794_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def test_batch_create_rejects_bad_descriptors(L):
    from paper_1009_0794_amd import _lib
    out = ctypes.c_void_p(7)
    d = (_lib.MeshDesc * 2)()
    for k in range(2):
        d[k] = _lib.MeshDesc(1, 3, 1, 1, (ctypes.c_float * 6)(0, 0, 0, 1, 1, 1), 8, 0, 0)
    assert L.ldni_batch_create(0, d, 7, None, ctypes.byref(out)) == 1 and out.value is None
    assert L.ldni_batch_create(2, d, 0, None, ctypes.byref(out)) == 1
    d[1].w = 0
    assert L.ldni_batch_create(2, d, 7, None, ctypes.byref(out)) == 1
    assert b"mesh 1" in L.ldni_last_error()
    d[1].w = 8
    d[0].tile_w, d[0].tile_h = 4, 4
    assert L.ldni_batch_create(2, d, 7, None, ctypes.byref(out)) == 1
    d[0].tile_w, d[0].tile_h = 0, 0
    d[0].bbox[3] = -1.0
    assert L.ldni_batch_create(2, d, 7, None, ctypes.byref(out)) == 1
    L.ldni_batch_free(None)
    v = _lib.AxisView()
    assert L.ldni_batch_axis(None, 0, 0, ctypes.byref(v)) == 1


def test_backward_rejects_bad_arguments(L):
    from paper_1009_0794_amd import _lib
    bb = (ctypes.c_float * 6)(0, 0, 0, 1, 1, 1)
    views = (_lib.AxisView * 3)()
    gd = (ctypes.c_void_p * 3)()
    gn = (ctypes.c_void_p * 3)()
    # NULL views, NULL grad_verts, mismatched resolution: rejected on the host
    assert L.ldni_backward(1, 3, 1, 1, bb, 8, 1, None, gd, gn, 1, None) == 1
    assert L.ldni_backward(1, 3, 1, 1, bb, 8, 1, views, gd, gn, None, None) == 1
    views[0].w = 16
    views[0].offsets = 1
    assert L.ldni_backward(1, 3, 1, 1, bb, 8, 1, views, gd, gn, 1, None) == 1
    assert L.ldni_backward(1, 3, 1, 1, bb, 0, 1, views, gd, gn, 1, None) == 1


def test_trim_with_nothing_cached(L):
    """ldni_trim releases the buffers kept between calls; with none kept it
    touches no device."""
    assert L.ldni_trim() == 0


def test_begin_rejects_misaligned_offsets(L):
    """Offsets are written with 16-byte stores: a buffer that is not 16-byte
    aligned is refused before any device work."""
    bb = (ctypes.c_float * 6)(0, 0, 0, 1, 1, 1)
    offs = (ctypes.c_void_p * 3)(0x1000 + 4, None, None)
    plan = ctypes.c_void_p(7)
    n = (ctypes.c_uint64 * 3)()
    assert L.ldni_sample_begin(0x2000, 3, 0x3000, 1, bb, 8, 1, offs, None, ctypes.byref(plan), n) == 1
    assert "aligned" in L.ldni_last_error().decode()
    assert plan.value is None


def _bool_call(L, a=True, b=True, op=0, eps=1e-5, axis=0, wa=8, wb=8, offsets=True, n=0, samples=True):
    from paper_1009_0794_amd import _lib
    def view(w):
        v = _lib.AxisView()
        v.w, v.n_samples = w, n
        v.offsets = 4096 if offsets else None
        if samples:
            v.depth = v.normal = v.tri = 8192
        return v
    va, vb = view(wa), view(wb)
    out = ctypes.c_void_p(123)
    rc = L.ldni_boolean(ctypes.byref(va) if a else None, ctypes.byref(vb) if b else None, op, eps,
                        axis, None, ctypes.byref(out))
    return rc, out.value


@pytest.mark.parametrize("kw", [
    dict(a=False), dict(b=False), dict(op=-1), dict(op=3), dict(eps=-1e-5), dict(eps=float("nan")),
    dict(eps=float("inf")), dict(axis=3), dict(axis=-1), dict(wa=8, wb=9), dict(wa=0, wb=0),
    dict(wa=16385, wb=16385), dict(offsets=False), dict(n=5, samples=False), dict(n=2 ** 32),
])
def test_boolean_invalid_arguments_rejected_on_host(L, kw):
    """ldni_boolean (Sec. 4.1) checks its arguments before any device work
    (the fake device pointers here are never dereferenced)."""
    rc, out = _bool_call(L, **kw)
    assert rc == 1
    assert out is None
    assert L.ldni_last_error().decode()


def test_finish_rgb8_rejects_null_plan(L):
    """ldni_sample_finish_rgb8 (Sec. 3 approximate normals) checks its
    arguments on the host."""
    arr = (ctypes.c_void_p * 3)()
    assert L.ldni_sample_finish_rgb8(None, arr, arr, arr) == 1
    assert L.ldni_sample_finish_rgb8(None, None, None, None) == 1


def _nodes_call(L, views=True, ws=(8, 8, 8), offsets=True, n=0, depth=True, bbox=(0, 0, 0, 1, 1, 1),
                bits=True, n_words=None):
    from paper_1009_0794_amd import _lib
    arr = (_lib.AxisView * 3)()
    for a in range(3):
        arr[a].w, arr[a].n_samples = ws[a], n
        arr[a].offsets = 4096 if offsets else None
        arr[a].depth = 8192 if depth else None
    bb = (ctypes.c_float * 6)(*bbox)
    need = ctypes.c_uint64()
    L.ldni_node_words(max(1, min(ws[0], 16384)), ctypes.byref(need))
    nw = need.value if n_words is None else n_words
    stats = (ctypes.c_uint64 * 2)(7, 7)
    rc = L.ldni_classify_nodes(arr if views else None, bb, 0x10000 if bits else None, nw, stats, None)
    return rc, list(stats)


@pytest.mark.parametrize("kw", [
    dict(views=False), dict(bits=False), dict(ws=(8, 8, 9)), dict(ws=(0, 0, 0)),
    dict(ws=(8193, 8193, 8193)), dict(offsets=False), dict(n=5, depth=False), dict(n=2 ** 32),
    dict(bbox=(0, 0, 0, 1, 0, 1)), dict(bbox=(0, 0, float("nan"), 1, 1, 1)),
    dict(bbox=(0, 0, 0, 1, 1, float("inf"))), dict(n_words=1024 - 1),
])
def test_classify_nodes_invalid_arguments_rejected_on_host(L, kw):
    """ldni_classify_nodes (Definition 3; Sec. 5.1 step 1) checks its
    arguments before any device work (the fake device pointers here are
    never dereferenced) and leaves the totals untouched."""
    rc, stats = _nodes_call(L, **kw)
    assert rc == 1
    assert stats == [7, 7]
    assert L.ldni_last_error().decode()


def test_node_words(L):
    """Bricks of 32^3 nodes, 1024 words each, ceil(w/32) per axis."""
    n = ctypes.c_uint64()
    for w, nb in ((1, 1), (32, 1), (33, 2), (2048, 64), (8192, 256)):
        assert L.ldni_node_words(w, ctypes.byref(n)) == 0
        assert n.value == nb ** 3 * 1024
    assert L.ldni_node_words(0, ctypes.byref(n)) == 1 and n.value == 0
    assert L.ldni_node_words(8193, ctypes.byref(n)) == 1 and n.value == 0
    assert L.ldni_node_words(8, None) == 1


def _offset_call(L, views=True, ws=(8, 8, 8), offsets=True, n=0, arrays=True, bbox=(0, 0, 0, 1, 1, 1),
                 r=0.1, eps=1e-5, out=True):
    from paper_1009_0794_amd import _lib
    arr = (_lib.AxisView * 3)()
    for a in range(3):
        arr[a].w, arr[a].n_samples = ws[a], n
        arr[a].offsets = 4096 if offsets else None
        if arrays:
            arr[a].depth = arr[a].normal = arr[a].tri = 8192
    bb = (ctypes.c_float * 6)(*bbox)
    res = ctypes.c_void_p(123)
    rc = L.ldni_offset(arr if views else None, bb, r, eps, None, ctypes.byref(res) if out else None)
    return rc, res.value


@pytest.mark.parametrize("kw", [
    dict(views=False), dict(out=False), dict(r=0.0), dict(r=float("nan")), dict(r=float("inf")),
    dict(eps=-1.0), dict(eps=float("nan")), dict(ws=(8, 9, 8)), dict(ws=(0, 0, 0)),
    dict(ws=(16385, 16385, 16385)), dict(offsets=False), dict(n=5, arrays=False), dict(n=2 ** 32),
    dict(n=2 ** 29), dict(bbox=(0, 0, 0, 1, 1, 0)), dict(bbox=(0, float("inf"), 0, 1, 1, 1)),
])
def test_offset_invalid_arguments_rejected_on_host(L, kw):
    """ldni_offset (Sec. 4.2) checks its arguments before any device work
    (the fake device pointers here are never dereferenced)."""
    rc, res = _offset_call(L, **kw)
    assert rc == 1
    assert res is None or not kw.get("out", True)
    assert L.ldni_last_error().decode()


def test_rgb8_option_only_where_declared(L):
    """LDNI_NORMAL_RGB8 (256) is an option of ldni_sample and the batch
    calls; ldni_sample_begin rejects it as an axis bit."""
    offs = (ctypes.c_void_p * 3)(1, 1, 1)
    n = (ctypes.c_uint64 * 3)()
    plan = ctypes.c_void_p()
    bb = (ctypes.c_float * 6)(0, 0, 0, 1, 1, 1)
    assert L.ldni_sample_begin(1, 3, 1, 1, bb, 8, 256 | 7, offs, None, ctypes.byref(plan), n) == 1


def test_axis_view_layout_matches_the_header():
    """The ctypes view has the header's eight fields in order (the last one
    the 8-bit normal codes)."""
    from paper_1009_0794_amd import _lib
    names = [f[0] for f in _lib.AxisView._fields_]
    assert names == ["w", "max_layers", "n_samples", "offsets", "depth", "normal", "tri", "normal_rgb8"]
    assert ctypes.sizeof(_lib.AxisView) == 4 + 4 + 8 + 5 * 8
    hdr = open(os.path.join(ROOT, "include", "ldni.h")).read()
    body = hdr[hdr.index("typedef struct {\n  int32_t w;"):hdr.index("} ldni_axis_view;")]
    fields = [m.group(1) for l in body.splitlines()
              for m in [re.match(r"\s*(?:const\s+)?\w+\s*\*?\s*(\w+);", l)] if m]
    assert fields == names, fields
