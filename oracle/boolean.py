"""TEST INFRASTRUCTURE ONLY: CPU oracle for Boolean operations on two LDNIs.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product library shares no code with it.

Method (Sec. 4.1 and Fig. 5 of the paper): in every pixel, the samples of a
solid bound its 1D volumes, read as consecutive pairs (enter, exit).  The
segments of A are sliced by the samples of B that fall inside them; then
  union         the slices of A outside B, together with B's segments;
  intersection  the slices of A inside B;
  difference    the slices of A outside B, and an end point that comes from
                B has its normal reversed.
Sec. 4.1.1 then removes every resulting 1D volume thinner than eps
(eps = 1e-5 in the paper, for single-precision depths).

Readings where the paper is silent:
  R1  A pixel with an odd sample count: its last, unpaired sample bounds no
      segment and is ignored.
  R2  Result pieces that touch (one ends at the depth where the next starts)
      form one volume: the result is the closure of the set where the
      operation holds, so no zero-thickness gap or sliver survives.
  R3  A result end point at depth d takes A's first sample at depth d if A
      has one there, else B's first sample at d.
  R4  A volume is removed when its thickness, (double)exit - (double)enter,
      is below eps or zero.
  R5  Output triangle ids: A's id t stays t; B's id t becomes -1 - t.
Depths, normals and ids of kept samples are copies of the inputs (a B
normal reversed for the difference), so results are exact.

``boolean`` loops over pixels in Python (small grids); ``boolean_c`` runs the
same steps in plain C (``boolean_oracle.c``) for whole large images.  The
pins run on both.
"""
from __future__ import annotations

import numpy as np

from . import AxisLDNI

UNION, INTERSECTION, DIFFERENCE = 0, 1, 2
OPS = {"union": UNION, "intersection": INTERSECTION, "difference": DIFFERENCE}


def _segments(d):
    """(enter depth, exit depth) of each consecutive pair (R1)."""
    n = len(d) // 2 * 2
    return [(float(d[i]), float(d[i + 1])) for i in range(0, n, 2)]


def _inside(segs, z):
    return any(s < z < e for s, e in segs)


def boolean_pixel(da, db, op, eps):
    """Result of one pixel as a list of (solid, sample index, reversed):
    solid 0 = A, 1 = B; the samples in depth order."""
    sa, sb = _segments(da), _segments(db)
    used_b = [float(db[j]) for j in range(len(db) // 2 * 2)]
    # slice A's segments by B's samples strictly inside them
    pieces = []
    for a0, a1 in sa:
        cuts = sorted({z for z in used_b if a0 < z < a1})
        pts = [a0] + cuts + [a1]
        pieces += [(pts[k], pts[k + 1]) for k in range(len(pts) - 1)]
    # classify the slices against B at their midpoints
    inside_b = [_inside(sb, 0.5 * (s + e)) for s, e in pieces]
    if op == UNION:
        keep = [p for p, ib in zip(pieces, inside_b) if not ib] + list(sb)
    elif op == INTERSECTION:
        keep = [p for p, ib in zip(pieces, inside_b) if ib]
    elif op == DIFFERENCE:
        keep = [p for p, ib in zip(pieces, inside_b) if not ib]
    else:
        raise ValueError("op must be UNION, INTERSECTION or DIFFERENCE")
    # merge pieces that overlap or touch (R2)
    keep.sort()
    vols = []
    for s, e in keep:
        if vols and s <= vols[-1][1]:
            vols[-1][1] = max(vols[-1][1], e)
        else:
            vols.append([s, e])
    # small interval removal (Sec. 4.1.1, R4)
    vols = [(s, e) for s, e in vols if e - s > 0.0 and e - s >= eps]
    na, nb = len(da) // 2 * 2, len(db) // 2 * 2

    def sample_at(z):  # R3
        for i in range(na):
            if float(da[i]) == z:
                return (0, i, False)
        for j in range(nb):
            if float(db[j]) == z:
                return (1, j, op == DIFFERENCE)
        raise AssertionError("a result end point is not a sample")

    out = []
    for s, e in vols:
        out += [sample_at(s), sample_at(e)]
    return out


def boolean(a: AxisLDNI, b: AxisLDNI, op, eps=1e-5) -> AxisLDNI:
    """Boolean operation of two LDNIs of one axis sampled on the same grid."""
    if isinstance(op, str):
        op = OPS[op]
    if a.w != b.w:
        raise ValueError("both LDNIs must have the same resolution")
    w = a.w
    offsets = np.zeros(w * w + 1, dtype=np.uint32)
    depth, normal, tri = [], [], []
    for p in range(w * w):
        ia, ja = int(a.offsets[p]), int(a.offsets[p + 1])
        ib, jb = int(b.offsets[p]), int(b.offsets[p + 1])
        res = boolean_pixel(a.depth[ia:ja], b.depth[ib:jb], op, eps)
        for solid, k, rev in res:
            src, base = (a, ia) if solid == 0 else (b, ib)
            depth.append(src.depth[base + k])
            n = np.asarray(src.normal[base + k], dtype=np.float32)
            normal.append(-n if rev else n)
            t = int(src.tri[base + k])
            tri.append(t if solid == 0 else -1 - t)
        offsets[p + 1] = offsets[p] + len(res)
    n = int(offsets[-1])
    return AxisLDNI(w=w, offsets=offsets,
                    depth=np.asarray(depth, dtype=np.float32).reshape(n),
                    normal=np.asarray(normal, dtype=np.float32).reshape(n, 3),
                    tri=np.asarray(tri, dtype=np.int32).reshape(n))


def boolean_c(a: AxisLDNI, b: AxisLDNI, op, eps=1e-5) -> AxisLDNI:
    """``boolean`` evaluated by the plain C restatement of the same steps."""
    import ctypes

    from . import _load
    if isinstance(op, str):
        op = OPS[op]
    if a.w != b.w:
        raise ValueError("both LDNIs must have the same resolution")
    lib = _load()
    w = a.w
    arrs = []
    for x in (a, b):
        arrs += [np.ascontiguousarray(x.offsets, np.uint32), np.ascontiguousarray(x.depth, np.float32),
                 np.ascontiguousarray(np.asarray(x.normal, np.float32).reshape(-1, 3)),
                 np.ascontiguousarray(x.tri, np.int32)]
    po = ctypes.POINTER(ctypes.c_uint32)()
    pd = ctypes.POINTER(ctypes.c_float)()
    pn = ctypes.POINTER(ctypes.c_float)()
    pt = ctypes.POINTER(ctypes.c_int32)()
    n = ctypes.c_uint64()
    rc = lib.oracle_boolean(w * w, *[q.ctypes.data for q in arrs], int(op), float(eps), ctypes.byref(po),
                            ctypes.byref(pd), ctypes.byref(pn), ctypes.byref(pt), ctypes.byref(n))
    if rc != 0:
        raise RuntimeError(f"oracle_boolean failed ({rc})")
    k = int(n.value)
    try:
        res = AxisLDNI(w=w, offsets=np.ctypeslib.as_array(po, (w * w + 1,)).copy(),
                       depth=np.ctypeslib.as_array(pd, (max(k, 1),))[:k].copy(),
                       normal=np.ctypeslib.as_array(pn, (max(k, 1) * 3,))[:3 * k].reshape(k, 3).copy(),
                       tri=np.ctypeslib.as_array(pt, (max(k, 1),))[:k].copy())
    finally:
        lib.oracle_boolean_free(po, pd, pn, pt)
    return res
