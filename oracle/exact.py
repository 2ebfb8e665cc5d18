"""TEST INFRASTRUCTURE ONLY: a rational-arithmetic micro-oracle for LDNI
sampling on tiny meshes.

It evaluates the ray-casting definition of an LDI/LDNI pixel (Sec. 2,
Definitions 1-2: every intersection of the ray through the pixel centre with
the surface, faces parallel to the ray excluded, depths ascending) with
``fractions.Fraction`` so that every sign and every depth is exact.  Only the
pixel-centre coordinates and the ray-frame translation are rounded, to float32,
exactly as the C oracle defines them (``ldni_oracle.h``), so that ties on
edges and vertices are decided on the same points.  Pure Python loops: use
it for meshes of a few dozen triangles and w up to about 16.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

AXES = "xyz"


def round_f32(q: Fraction) -> Fraction:
    """Round a rational to the nearest float32 (ties to even), subnormals
    included; returns the float32 value as a Fraction."""
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)                 # subnormal range keeps the -126 exponent
    ulp = Fraction(2) ** (e - 23)
    m = a / ulp                      # significand in units of ulp
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * ulp
    if r >= Fraction(2) ** 128:
        raise OverflowError("float32 overflow")
    return sign * r


def _sgn(x) -> int:
    return (x > 0) - (x < 0)


def pixel_centres(lo: float, hi: float, w: int):
    """Centre of pixel i: the float64 evaluation lo + (i + 0.5) * h with
    h = (hi - lo) / w, rounded once to float32 (Sec. 3, pixel centres)."""
    lo = float(np.float32(lo))
    hi = float(np.float32(hi))
    h = (hi - lo) / w
    return [round_f32(Fraction(lo + (i + 0.5) * h)) for i in range(w)]


def edge_sign(xu, xv, yu, yv) -> int:
    """Exact sign of X'_u*Y'_v - X'_v*Y'_u; a zero is resolved by moving the
    ray to (+eps, +eps^2): first X'_v - Y'_v, then Y'_u - X'_u."""
    s = _sgn(xu * yv - xv * yu)
    if s:
        return s
    s = _sgn(xv - yv)
    if s:
        return s
    return _sgn(yu - xu)


def sample_pixel(verts, tris, axis: int, cu: Fraction, cv: Fraction, lo_a: float):
    """All hits of one ray: list of (exact depth from lo_a, triangle id),
    sorted by (depth, id)."""
    u, v = (axis + 1) % 3, (axis + 2) % 3
    lo_a = Fraction(float(np.float32(lo_a)))
    hits = []
    for t, (ia, ib, ic) in enumerate(tris):
        P = [[Fraction(float(c)) for c in verts[k]] for k in (ia, ib, ic)]
        tu = [round_f32(p[u] - cu) for p in P]
        tv = [round_f32(p[v] - cv) for p in P]
        s_ab = edge_sign(tu[0], tv[0], tu[1], tv[1])
        s_bc = edge_sign(tu[1], tv[1], tu[2], tv[2])
        s_ca = edge_sign(tu[2], tv[2], tu[0], tv[0])
        if s_ab == 0 or not (s_ab == s_bc == s_ca):
            continue
        e_ab = tu[0] * tv[1] - tv[0] * tu[1]
        e_bc = tu[1] * tv[2] - tv[1] * tu[2]
        e_ca = tu[2] * tv[0] - tv[2] * tu[0]
        den = e_ab + e_bc + e_ca
        # barycentric weights of A, B, C are E_BC, E_CA, E_AB over den
        z = (e_bc * P[0][axis] + e_ca * P[1][axis] + e_ab * P[2][axis]) / den
        hits.append((z - lo_a, t))
    hits.sort()
    return hits


def sample(verts, tris, bbox, w: int, axes="xyz"):
    """Exact LDNI of a tiny mesh: ``{axis: [[(depth, tri), ...] per pixel]}``
    with pixels in the order p = j*w + i."""
    verts = np.asarray(verts, dtype=np.float32)
    tris = np.asarray(tris, dtype=np.int64)
    out = {}
    for a in [AXES.index(c) for c in axes] if isinstance(axes, str) else axes:
        u, v = (a + 1) % 3, (a + 2) % 3
        cus = pixel_centres(bbox[u], bbox[3 + u], w)
        cvs = pixel_centres(bbox[v], bbox[3 + v], w)
        out[a] = [sample_pixel(verts, tris, a, cus[i], cvs[j], bbox[a])
                  for j in range(w) for i in range(w)]
    return out


def face_normal(verts, tri) -> tuple:
    """Exact unnormalised face normal (B-A) x (C-A)."""
    A, B, C = ([Fraction(float(c)) for c in verts[k]] for k in tri)
    e1 = [B[k] - A[k] for k in range(3)]
    e2 = [C[k] - A[k] for k in range(3)]
    return (e1[1] * e2[2] - e1[2] * e2[1],
            e1[2] * e2[0] - e1[0] * e2[2],
            e1[0] * e2[1] - e1[1] * e2[0])
