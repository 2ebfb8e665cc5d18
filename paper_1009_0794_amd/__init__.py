"""MI355X (gfx950) Layered Depth-Normal Image sampling.

Python binding of the C ABI in ``include/ldni.h``: it marshals torch device
tensors and the current HIP stream into the library; every step of the
sampling runs in the library's HIP kernels.  There is no CPU fallback: if
``libldni.so`` is missing, every entry point raises.

``sample`` builds the LDNIs of a closed triangle mesh (Wang & Chen, Sec. 2
Definitions 1-3, built by rasterisation in Sec. 3): per axis, every
intersection of the w x w pixel-centre rays with the mesh as a (depth, unit
face normal) sample, in compact per-pixel rows sorted by depth.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Dict

from . import _lib
from ._lib import LDNIError

__all__ = ["LDNI", "LDNIError", "sample", "ldni_sample", "ldni_result_axis", "ldni_free", "ldni_trim",
           "ldni_sample_begin", "ldni_sample_finish", "ldni_plan_free", "ldni_status_string",
           "set_tile_shape", "axis_mask", "library_path", "profile_enable", "profile_read",
           "ldni_backward", "sample_diff", "LDNISample", "Batch", "sample_batch", "ldni_boolean",
           "boolean", "BOOLEAN_OPS", "ldni_classify_nodes", "classify_nodes", "node_words",
           "ldni_offset", "offset"]

AXES = "xyz"
library_path = _lib.LIB_PATH


NORMAL_RGB8 = 256  # option bit of the axis mask: 8-bit normal codes (LDNI_NORMAL_RGB8)


def _normals_flag(normals: str) -> int:
    if normals not in ("f32", "rgb8"):
        raise ValueError("normals must be 'f32' or 'rgb8'")
    return NORMAL_RGB8 if normals == "rgb8" else 0


def axis_mask(axes) -> int:
    if isinstance(axes, int):
        return axes
    m = 0
    for c in axes:
        m |= 1 << AXES.index(c)
    return m


def _torch():
    import torch
    return torch


@dataclass
class LDNI:
    """One axis of an LDNI in compact rows: the samples of pixel
    p = j*w + i are ``[offsets[p], offsets[p+1])`` (offsets hold u32 values in
    an int32 tensor)."""
    axis: int
    w: int
    max_layers: int
    offsets: "torch.Tensor"   # int32 [w*w+1] (u32 bit patterns)
    depth: "torch.Tensor"     # float32 [n]
    normal: "torch.Tensor"    # float32 [n, 3]
    tri: "torch.Tensor"       # int32 [n]

    @property
    def n(self) -> int:
        return int(self.depth.shape[0])

    def offsets64(self):
        return self.offsets.to(_torch().int64) & 0xFFFFFFFF

    def counts(self):
        return self.offsets64().diff()


def _check_mesh(verts, tris):
    torch = _torch()
    if not (verts.is_cuda and tris.is_cuda):
        raise ValueError("verts and tris must be device tensors")
    if verts.dtype != torch.float32 or tris.dtype != torch.int32:
        raise TypeError("verts must be float32 [V,3], tris int32 [T,3]")
    if verts.dim() != 2 or verts.shape[1] != 3 or tris.dim() != 2 or tris.shape[1] != 3:
        raise ValueError("verts must be [V,3], tris [T,3]")
    return verts.contiguous(), tris.contiguous()


def _bbox(bbox):
    b = (ctypes.c_float * 6)(*[float(x) for x in bbox])
    return b


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def ldni_sample_begin(verts, tris, bbox, w, axes="xyz"):
    """First half of sampling: returns (plan handle, offsets tensors by axis,
    sample counts by axis)."""
    torch = _torch()
    verts, tris = _check_mesh(verts, tris)
    mask = axis_mask(axes)
    L = _lib.lib()
    dev = verts.device
    offs = {}
    optr = (ctypes.c_void_p * 3)()
    for a in range(3):
        if (mask >> a) & 1:
            offs[a] = torch.empty(int(w) * int(w) + 1, dtype=torch.int32, device=dev)
            optr[a] = offs[a].data_ptr()
    plan = ctypes.c_void_p()
    n = (ctypes.c_uint64 * 3)()
    bb = _bbox(bbox)
    _lib.check(L.ldni_sample_begin(verts.data_ptr(), verts.shape[0], tris.data_ptr(),
                                   tris.shape[0], bb, int(w), mask, optr, _stream(dev),
                                   ctypes.byref(plan), n))
    return plan, offs, [int(x) for x in n]


def ldni_sample_finish(plan, depth, normal, tri, rgb8=False):
    """Second half: writes the samples into the given tensors (dicts by axis)
    and releases the plan.  With rgb8, ``normal`` holds int32 [n] tensors that
    receive the 8-bit normal codes (``ldni_sample_finish_rgb8``)."""
    L = _lib.lib()
    d, nm, t = (ctypes.c_void_p * 3)(), (ctypes.c_void_p * 3)(), (ctypes.c_void_p * 3)()
    for a in depth:
        d[a], nm[a], t[a] = depth[a].data_ptr(), normal[a].data_ptr(), tri[a].data_ptr()
    fn = L.ldni_sample_finish_rgb8 if rgb8 else L.ldni_sample_finish
    _lib.check(fn(plan, d, nm, t))


def ldni_plan_free(plan):
    _lib.lib().ldni_plan_free(plan)


def sample(verts, tris, bbox, w: int, axes="xyz", normals="f32") -> Dict[int, LDNI]:
    """LDNIs of a mesh as torch tensors on the mesh's device.

    verts float32 [V,3] and tris int32 [T,3] (counter-clockwise seen from
    outside) on a HIP device; bbox = (xlo, ylo, zlo, xhi, yhi, zhi) on the host;
    returns ``{axis: LDNI}`` for the requested axes.  normals="rgb8" stores the
    paper's approximate normals: ``normal`` is then an int32 [n] tensor of
    packed 8-bit codes (x | y << 8 | z << 16, component ~ byte / 127.5 - 1)."""
    if normals not in ("f32", "rgb8"):
        raise ValueError("normals must be 'f32' or 'rgb8'")
    rgb8 = normals == "rgb8"
    torch = _torch()
    verts, tris = _check_mesh(verts, tris)
    plan, offs, n = ldni_sample_begin(verts, tris, bbox, w, axes)
    L = _lib.lib()
    ml = (ctypes.c_uint32 * 3)()
    try:
        _lib.check(L.ldni_plan_max_layers(plan, ml))
        dev = verts.device
        depth, normal, tri = {}, {}, {}
        for a in offs:
            depth[a] = torch.empty(n[a], dtype=torch.float32, device=dev)
            normal[a] = (torch.empty(n[a], dtype=torch.int32, device=dev) if rgb8 else
                         torch.empty((n[a], 3), dtype=torch.float32, device=dev))
            tri[a] = torch.empty(n[a], dtype=torch.int32, device=dev)
    except BaseException:
        ldni_plan_free(plan)
        raise
    ldni_sample_finish(plan, depth, normal, tri, rgb8=rgb8)
    return {a: LDNI(a, int(w), int(ml[a]), offs[a], depth[a], normal[a], tri[a]) for a in offs}


def _view(l: LDNI) -> _lib.AxisView:
    """An input view; an LDNI with 8-bit normal codes passes no float normals
    (the operations that read normals then reject it)."""
    ptr = lambda t: None if t is None else t.data_ptr()
    normal = l.normal if (l.normal is not None and l.normal.dtype == _torch().float32) else None
    return _lib.AxisView(int(l.w), int(max(l.max_layers, 0)), int(l.tri.shape[0]),
                         l.offsets.data_ptr(), ptr(l.depth), ptr(normal), l.tri.data_ptr())


def ldni_backward(verts, tris, bbox, w: int, ldnis: Dict[int, LDNI], grad_depth=None,
                  grad_normal=None, grad_verts=None, no_alloc=False):
    """Adds to ``grad_verts`` (created as zeros if None) the vertex gradient of
    sum(gd * depth) + sum(gn . normal) over the samples of ``ldnis``;
    ``grad_depth``/``grad_normal`` map axis -> float32 device tensors [n] and
    [n, 3] (missing axes are zero).  Returns grad_verts.  With ``no_alloc``
    the call goes to ``ldni_backward_noalloc`` (no device allocation by the
    library; at most 262,144 triangles)."""
    torch = _torch()
    verts, tris = _check_mesh(verts, tris)
    if grad_verts is None:
        grad_verts = torch.zeros_like(verts)
    grad_depth = grad_depth or {}
    grad_normal = grad_normal or {}
    views = (_lib.AxisView * 3)()
    gd = (ctypes.c_void_p * 3)()
    gn = (ctypes.c_void_p * 3)()
    keep = []
    mask = 0
    for a, l in ldnis.items():
        mask |= 1 << a
        views[a] = _view(l)
        n = int(l.tri.shape[0])
        for src, dst, shape in ((grad_depth, gd, (n,)), (grad_normal, gn, (n, 3))):
            g = src.get(a)
            if g is not None:
                g = g.to(device=verts.device, dtype=torch.float32).contiguous()
                if tuple(g.shape) != shape:
                    raise ValueError(f"gradient of axis {a} has shape {tuple(g.shape)}, expected {shape}")
                keep.append(g)
                dst[a] = g.data_ptr()
    if mask == 0:
        return grad_verts
    if not (grad_verts.is_contiguous() and grad_verts.dtype == torch.float32
            and tuple(grad_verts.shape) == tuple(verts.shape)):
        raise ValueError("grad_verts must be a contiguous float32 tensor shaped like verts")
    fn = _lib.lib().ldni_backward_noalloc if no_alloc else _lib.lib().ldni_backward
    _lib.check(fn(verts.data_ptr(), verts.shape[0], tris.data_ptr(), tris.shape[0], _bbox(bbox), int(w), mask,
                  views, gd, gn, grad_verts.data_ptr(), _stream(verts.device)))
    return grad_verts


def _autograd_function():
    torch = _torch()

    class LDNISample(torch.autograd.Function):
        """Differentiable sampling: outputs (depth, normal) per requested axis,
        then (offsets, tri, max_layers) per axis, the latter not
        differentiable.  The backward pass is the library's ldni_backward."""

        @staticmethod
        def forward(ctx, verts, tris, bbox, w, axes):
            res = sample(verts, tris, bbox, w, axes)
            order = sorted(res)
            ctx.order = order
            ctx.bbox = tuple(bbox)
            ctx.w = int(w)
            ctx.save_for_backward(verts, tris, *[res[a].offsets for a in order],
                                  *[res[a].tri for a in order])
            outs = []
            for a in order:
                outs += [res[a].depth, res[a].normal]
            extra = []
            for a in order:
                extra += [res[a].offsets, res[a].tri,
                          torch.tensor(res[a].max_layers, dtype=torch.int64)]
            ctx.mark_non_differentiable(*extra)
            return tuple(outs + extra)

        @staticmethod
        def backward(ctx, *grads):
            saved = ctx.saved_tensors
            verts, tris = saved[0], saved[1]
            k_ax = len(ctx.order)
            ldnis = {a: LDNI(a, ctx.w, 0, saved[2 + i], None, None, saved[2 + k_ax + i])
                     for i, a in enumerate(ctx.order)}
            gd, gn = {}, {}
            for k, a in enumerate(ctx.order):
                if grads[2 * k] is not None:
                    gd[a] = grads[2 * k]
                if grads[2 * k + 1] is not None:
                    gn[a] = grads[2 * k + 1]
            g = ldni_backward(verts.detach(), tris, ctx.bbox, ctx.w, ldnis, gd, gn)
            return g, None, None, None, None

    return LDNISample


_LDNISample = None


def LDNISample():
    """The torch.autograd.Function class behind ``sample_diff``."""
    global _LDNISample
    if _LDNISample is None:
        _LDNISample = _autograd_function()
    return _LDNISample


def sample_diff(verts, tris, bbox, w: int, axes="xyz") -> Dict[int, LDNI]:
    """Like ``sample`` but ``depth`` and ``normal`` carry gradients to
    ``verts`` (through ldni_backward)."""
    fn = LDNISample()
    outs = fn.apply(verts, tris, tuple(float(x) for x in bbox), int(w), axes)
    order = sorted(AXES.index(c) for c in axes) if isinstance(axes, str) else sorted(axes)
    k = len(order)
    res = {}
    for i, a in enumerate(order):
        off, tri, ml = outs[2 * k + 3 * i: 2 * k + 3 * i + 3]
        res[a] = LDNI(a, int(w), int(ml), off, outs[2 * i], outs[2 * i + 1], tri)
    return res


# ---- library-owned results -------------------------------------------------

class Result:
    """Owner of an ``ldni_result``; frees it when collected."""

    def __init__(self, handle: ctypes.c_void_p):
        self.handle = handle

    def view(self, axis: int) -> _lib.AxisView:
        v = _lib.AxisView()
        _lib.check(_lib.lib().ldni_result_axis(self.handle, int(axis), ctypes.byref(v)))
        return v

    def to_torch(self, axis: int, device=None) -> LDNI:
        """Copy one axis into new torch tensors (device-to-device)."""
        torch = _torch()
        dev = torch.device("cuda") if device is None else torch.device(device)
        return _copy_view(self.view(axis), axis, dev)

    def free(self):
        if self.handle:
            _lib.lib().ldni_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def ldni_sample(verts, tris, bbox, w: int, axes="xyz", stream=None, normals="f32") -> Result:
    """The one-call C ABI: the library allocates and owns the outputs.
    normals="rgb8" stores 8-bit normal codes (the views' normal_rgb8)."""
    verts, tris = _check_mesh(verts, tris)
    h = ctypes.c_void_p()
    st = _stream(verts.device) if stream is None else ctypes.c_void_p(stream)
    _lib.check(_lib.lib().ldni_sample(verts.data_ptr(), verts.shape[0], tris.data_ptr(),
                                      tris.shape[0], _bbox(bbox), int(w),
                                      axis_mask(axes) | _normals_flag(normals), st, ctypes.byref(h)))
    return Result(h)


BOOLEAN_OPS = {"union": 0, "intersection": 1, "difference": 2}


def ldni_boolean(a: LDNI, b: LDNI, op, eps: float = 1e-5, stream=None) -> Result:
    """The C ABI ``ldni_boolean``: Boolean operation (Sec. 4.1, small interval
    removal Sec. 4.1.1) of two LDNIs of one axis sampled on the same grid; the
    library owns the result, whose view ``a.axis`` holds it."""
    if isinstance(op, str):
        op = BOOLEAN_OPS[op]
    h = ctypes.c_void_p()
    st = _stream(a.depth.device) if stream is None else ctypes.c_void_p(stream)
    va, vb = _view(a), _view(b)
    _lib.check(_lib.lib().ldni_boolean(ctypes.byref(va), ctypes.byref(vb), int(op), float(eps),
                                       int(a.axis), st, ctypes.byref(h)))
    return Result(h)


def boolean(a: LDNI, b: LDNI, op, eps: float = 1e-5) -> LDNI:
    """``ldni_boolean`` with the result copied into new torch tensors."""
    r = ldni_boolean(a, b, op, eps)
    try:
        return _copy_view(r.view(a.axis), a.axis, a.depth.device)
    finally:
        r.free()


def node_words(w: int) -> int:
    """``ldni_node_words``: 32-bit words of the node bit volume at resolution w."""
    n = ctypes.c_uint64()
    _lib.check(_lib.lib().ldni_node_words(int(w), ctypes.byref(n)))
    return int(n.value)


def ldni_classify_nodes(ldnis, bbox, bits=None):
    """The C ABI ``ldni_classify_nodes`` (Definition 3; Sec. 5.1 step 1): the
    inside/outside bit of every node of the w^3 grid where the rays of the
    x-, y- and z-LDNI (``ldnis[0..2]``, sampled with ``bbox``) meet, by a
    two-of-three vote.  ``bits`` (int32 device tensor of ``node_words(w)``
    words, allocated if None) receives 32^3-node bricks; returns (bits,
    nodes inside, nodes whose three votes differ)."""
    torch = _torch()
    L = [ldnis[a] for a in range(3)]
    w = int(L[0].w)
    n = node_words(w)
    dev = L[0].depth.device
    if bits is None:
        bits = torch.empty(n, dtype=torch.int32, device=dev)
    elif bits.dtype != torch.int32 or not bits.is_contiguous() or bits.numel() < n or bits.device != dev:
        raise ValueError(f"bits must be a contiguous int32 tensor of at least {n} words on {dev}")
    views = (_lib.AxisView * 3)(*[_view(l) for l in L])
    bb = (ctypes.c_float * 6)(*[float(x) for x in bbox])
    stats = (ctypes.c_uint64 * 2)()
    _lib.check(_lib.lib().ldni_classify_nodes(views, bb, ctypes.c_void_p(bits.data_ptr()), n, stats,
                                              _stream(dev)))
    return bits, int(stats[0]), int(stats[1])


classify_nodes = ldni_classify_nodes


def ldni_offset(ldnis, bbox, r: float, eps: float = 1e-5) -> Result:
    """The C ABI ``ldni_offset`` (Sec. 4.2): the solid whose x-, y-, z-LDNIs are
    ``ldnis[0..2]`` (sampled with ``bbox``) offset by r, as the union with a
    sphere of radius r at every sample (r < 0: their difference); the library
    owns the three-axis result."""
    L = [ldnis[a] for a in range(3)]
    views = (_lib.AxisView * 3)(*[_view(l) for l in L])
    bb = (ctypes.c_float * 6)(*[float(x) for x in bbox])
    h = ctypes.c_void_p()
    _lib.check(_lib.lib().ldni_offset(views, bb, float(r), float(eps), _stream(L[0].depth.device),
                                      ctypes.byref(h)))
    return Result(h)


def offset(ldnis, bbox, r: float, eps: float = 1e-5) -> Dict[int, LDNI]:
    """``ldni_offset`` with the three axes copied into new torch tensors."""
    dev = ldnis[0].depth.device
    res = ldni_offset(ldnis, bbox, r, eps)
    try:
        return {a: _copy_view(res.view(a), a, dev) for a in range(3)}
    finally:
        res.free()


def _copy_view(v: _lib.AxisView, axis: int, device) -> LDNI:
    """Copies a view into new tensors; a view with 8-bit normal codes gives
    an int32 [n] ``normal`` tensor of the codes."""
    torch = _torch()
    n = int(v.n_samples)
    rgb8 = bool(v.normal_rgb8)
    out = LDNI(axis, int(v.w), int(v.max_layers),
               torch.empty(int(v.w) * int(v.w) + 1, dtype=torch.int32, device=device),
               torch.empty(n, dtype=torch.float32, device=device),
               (torch.empty(n, dtype=torch.int32, device=device) if rgb8 else
                torch.empty((n, 3), dtype=torch.float32, device=device)),
               torch.empty(n, dtype=torch.int32, device=device))
    H = _lib.hip()
    st = _stream(device)
    for dst, src, nbytes in ((out.offsets, v.offsets, 4 * out.offsets.numel()),
                             (out.depth, v.depth, 4 * n),
                             (out.normal, v.normal_rgb8 if rgb8 else v.normal, (4 if rgb8 else 12) * n),
                             (out.tri, v.tri, 4 * n)):
        if nbytes:
            rc = H.hipMemcpyAsync(dst.data_ptr(), src, nbytes, 3, st)
            if rc != 0:
                raise RuntimeError(f"hipMemcpyAsync failed ({rc})")
    return out


class Batch:
    """Many meshes sampled by one captured graph (``ldni_batch_*``).

    ``meshes``: sequence of (verts, tris, bbox, w) or (verts, tris, bbox, w,
    (tile_w, tile_h)) with device tensors, which must stay alive and at the
    same addresses; ``run()`` samples their current contents again."""

    def __init__(self, meshes, axes="xyz", normals="f32"):
        torch = _torch()
        flag = _normals_flag(normals)
        self._keep = []
        descs = (_lib.MeshDesc * len(meshes))()
        dev = None
        for k, m in enumerate(meshes):
            verts, tris, bbox, w = m[:4]
            tile = m[4] if len(m) > 4 and m[4] is not None else (0, 0)
            verts, tris = _check_mesh(verts, tris)
            dev = verts.device
            self._keep += [verts, tris]
            descs[k] = _lib.MeshDesc(verts.data_ptr(), verts.shape[0], tris.data_ptr(), tris.shape[0],
                                     (ctypes.c_float * 6)(*[float(x) for x in bbox]), int(w),
                                     int(tile[0]), int(tile[1]))
        self.device = dev if dev is not None else torch.device("cuda")
        self.n_meshes = len(meshes)
        self.mask = axis_mask(axes)
        self.handle = ctypes.c_void_p()
        _lib.check(_lib.lib().ldni_batch_create(len(meshes), descs, self.mask | flag, _stream(self.device),
                                                ctypes.byref(self.handle)))

    def run(self):
        _lib.check(_lib.lib().ldni_batch_run(self.handle, _stream(self.device)))

    def view(self, mesh: int, axis: int) -> _lib.AxisView:
        v = _lib.AxisView()
        _lib.check(_lib.lib().ldni_batch_axis(self.handle, int(mesh), int(axis), ctypes.byref(v)))
        return v

    def to_torch(self, mesh: int, axis: int) -> LDNI:
        return _copy_view(self.view(mesh, axis), axis, self.device)

    def free(self):
        if self.handle:
            _lib.lib().ldni_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def sample_batch(meshes, axes="xyz", tiles="auto", normals="f32") -> Batch:
    """Create (and run once) a batch; see ``Batch``.  With tiles="auto",
    meshes given without a tile shape get the autotuned one for their
    resolution and triangle density, tuned inside a batch where that table
    has the bucket (``autotune.batch_lookup``)."""
    if tiles == "auto":
        from . import autotune
        table, btable = autotune.load_table(), autotune.load_table(autotune.BATCH_TABLE_PATH)
        meshes = [tuple(m[:4]) + ((m[4] if len(m) > 4 and m[4] is not None
                                   else autotune.batch_lookup(int(m[3]), int(m[1].shape[0]), btable, table)),)
                  for m in meshes]
    return Batch(meshes, axes, normals)


def ldni_result_axis(result: Result, axis: int) -> _lib.AxisView:
    return result.view(axis)


def ldni_free(result: Result) -> None:
    result.free()


def ldni_trim() -> None:
    """Hand the device buffers the library keeps between calls back to the
    device (no call may be in flight)."""
    _lib.check(_lib.lib().ldni_trim())


def ldni_status_string(code: int) -> str:
    return _lib.lib().ldni_status_string(int(code)).decode()


def profile_enable(on: bool = True) -> None:
    """Start (clearing earlier records) or stop per-kernel HIP-event timing."""
    _lib.check(_lib.lib().ldni_profile_enable(1 if on else 0))


def profile_read() -> Dict[str, tuple]:
    """{kernel name: (launches, total milliseconds)} of the recorded launches."""
    L = _lib.lib()
    n = ctypes.c_int32()
    _lib.check(L.ldni_profile_read(None, 0, ctypes.byref(n)))
    arr = (_lib.KernelStat * max(1, n.value))()
    _lib.check(L.ldni_profile_read(arr, n.value, ctypes.byref(n)))
    return {arr[k].name.decode(): (int(arr[k].launches), float(arr[k].total_ms))
            for k in range(n.value)}


def set_tile_shape(tw: int, th: int) -> None:
    _lib.check(_lib.lib().ldni_set_tile_shape(int(tw), int(th)))
