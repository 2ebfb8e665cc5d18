"""TEST INFRASTRUCTURE ONLY: CPU oracle for offsetting a solid given by LDNIs.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product library shares no code with it.

Method (Sec. 4.2): the offset of a solid H by a distance r is approximated
by the Minkowski sum of H with a sphere of radius r: a sphere S of radius r
is centred at every depth-normal sample of H's LDNIs, S is itself sampled
into LDNIs on the same grid, and H is united with every such S (for an
inner offset, r < 0, every S of radius |r| is subtracted from H).  The
Boolean operations are those of Sec. 4.1 with small interval removal
(Sec. 4.1.1).

Readings where the paper is silent:
  OF1  The spheres sit at every sample of all three LDNIs.  The centre of a
       sample of the a-LDNI at pixel (iu, iv) is the point whose a-coordinate
       is lo_a + depth and whose other two coordinates are the pixel centres
       c_u[iu], c_v[iv] (float64 from the float32 values).
  OF2  A sphere's LDNI, on a ray of axis a through (c_u, c_v): with
       rho2 = (c_u - p_u)^2 + (c_v - p_v)^2 in float64, the ray is hit when
       rho2 < r^2 (a tangent ray is not), at z = p_a -/+ sqrt(r^2 - rho2)
       (enter, exit); depths f32(z - lo_a); the normal is ((x - p) / |r|) in
       float64 rounded to float32 (world order) for the union and its negation
       for the difference.
  OF3  All spheres are applied at once (a union of sets does not depend on
       order): per ray, the events are H's paired samples (an unpaired last
       sample is ignored, as Boolean reading B1) and the enter and exit of
       every sphere that hits the ray; events of equal float32 depth form one
       group; after a group, H's state is the parity of its samples so far and
       the spheres' state is "some sphere entered and not yet left"; the
       result state is H or S (union), H and not S (difference).  A group that
       changes the result state contributes one end point: its first event in
       the order H's samples (by index), then spheres by generating sample,
       a sphere's enter before its exit.  Volumes with (double)exit -
       (double)enter <= 0 or < eps are removed (Sec. 4.1.1).
  OF4  Generating samples are numbered g = 0, 1, ... over the x-, then the y-,
       then the z-LDNI, each in storage order.  A result sample from H keeps
       its triangle id; one from the sphere of sample g has id -1 - g.
Depths, normals and ids of kept H samples are copies; sphere samples are
computed as in OF2, so results are exact.
"""
from __future__ import annotations

import math

import numpy as np

from . import AxisLDNI, bbox_f32


def _centres(lo, hi, w):
    h = (float(hi) - float(lo)) / float(w)
    return (float(lo) + (np.arange(w, dtype=np.float64) + 0.5) * h).astype(np.float32).astype(np.float64)


def sphere_centres(L, bbox, w):
    """Centres (float64 [N,3], world order) of the spheres of all samples,
    numbered as OF4."""
    b = bbox_f32(bbox)
    out = []
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        cu, cv = _centres(b[u], b[3 + u], w), _centres(b[v], b[3 + v], w)
        ax = L[a]
        cnt = np.diff(ax.offsets.astype(np.int64))
        pix = np.repeat(np.arange(w * w), cnt)
        p = np.zeros((len(pix), 3))
        p[:, a] = b[a] + ax.depth.astype(np.float64)
        p[:, u] = cu[pix % w]
        p[:, v] = cv[pix // w]
        out.append(p)
    return np.concatenate(out) if out else np.zeros((0, 3))


def _ray_events(a, cu_val, cv_val, centres, r, lo_a, union, order=None):
    """The spheres hitting one ray: list of (depth, g, is_exit, normal).
    ``order`` (optional) lists the spheres sorted by their u coordinate, so
    only those with |p_u - c_u| <= r are tested."""
    u, v = (a + 1) % 3, (a + 2) % 3
    if order is None:
        cand = np.arange(len(centres))
    else:
        srt, pu = order
        lo_i = np.searchsorted(pu, cu_val - r, side="left")
        hi_i = np.searchsorted(pu, cu_val + r, side="right")
        cand = np.sort(srt[lo_i:hi_i])
    du = cu_val - centres[cand, u]
    dv = cv_val - centres[cand, v]
    rho2 = du * du + dv * dv
    sel = np.nonzero(rho2 < r * r)[0]
    hit = cand[sel]
    du, dv, rho2 = du[sel], dv[sel], rho2[sel]
    ev = []
    sign = 1.0 if union else -1.0
    for q, g in enumerate(hit):
        t = math.sqrt(r * r - rho2[q])
        pa = centres[g, a]
        for is_exit, z in ((0, pa - t), (1, pa + t)):
            n = np.zeros(3)
            n[u] = du[q] / r
            n[v] = dv[q] / r
            n[a] = (z - pa) / r
            ev.append((np.float32(z - lo_a), int(g), is_exit, (sign * n).astype(np.float32)))
    return ev


def offset_pixel(h_depth, h_normal, h_tri, sphere_events, union, eps):
    """Result of one ray: list of (depth, normal, id)."""
    n_h = len(h_depth) // 2 * 2
    events = []  # (depth, order key, kind, payload)
    for k in range(n_h):
        events.append((float(h_depth[k]), (0, k, 0), "h", k))
    for d, g, is_exit, nrm in sphere_events:
        events.append((float(d), (1, g, is_exit), "s", (d, g, is_exit, nrm)))
    events.sort(key=lambda e: (e[0], e[1]))
    out = []
    in_h, depth_s, in_r = False, 0, False
    k = 0
    while k < len(events):
        d = events[k][0]
        first = events[k]
        while k < len(events) and events[k][0] == d:
            e = events[k]
            if e[2] == "h":
                in_h = not in_h
            else:
                depth_s += -1 if e[3][2] else 1
            k += 1
        now = (in_h or depth_s > 0) if union else (in_h and depth_s == 0)
        if now != in_r:
            if first[2] == "h":
                q = first[3]
                out.append((np.float32(h_depth[q]), np.asarray(h_normal[q], np.float32), int(h_tri[q])))
            else:
                dd, g, _, nrm = first[3]
                out.append((np.float32(dd), nrm, -1 - g))
            in_r = now
    kept = []
    for s in range(0, len(out) // 2 * 2, 2):
        t = float(out[s + 1][0]) - float(out[s][0])
        if t > 0.0 and t >= eps:
            kept += [out[s], out[s + 1]]
    return kept


def offset(L, bbox, w, r, eps=1e-5):
    """Offset of the solid whose x-, y-, z-LDNIs are L[0..2] (sampled on
    ``bbox`` at resolution w) by r (r > 0 outward by union, r < 0 inward by
    difference).  Returns {axis: AxisLDNI}."""
    if r == 0:
        raise ValueError("r must not be zero")
    union = r > 0
    rr = abs(float(np.float32(r)))
    b = bbox_f32(bbox)
    centres = sphere_centres(L, bbox, w)
    res = {}
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        cu, cv = _centres(b[u], b[3 + u], w), _centres(b[v], b[3 + v], w)
        ax = L[a]
        srt = np.argsort(centres[:, u], kind="stable")
        order = (srt, centres[srt, u])
        offsets = np.zeros(w * w + 1, np.uint32)
        dep, nrm, tri = [], [], []
        for p in range(w * w):
            o0, o1 = int(ax.offsets[p]), int(ax.offsets[p + 1])
            ev = _ray_events(a, cu[p % w], cv[p // w], centres, rr, b[a], union, order)
            got = offset_pixel(ax.depth[o0:o1], ax.normal[o0:o1], ax.tri[o0:o1], ev, union, eps)
            for d, n, t in got:
                dep.append(d)
                nrm.append(n)
                tri.append(t)
            offsets[p + 1] = offsets[p] + len(got)
        n = int(offsets[-1])
        res[a] = AxisLDNI(w=w, offsets=offsets, depth=np.asarray(dep, np.float32).reshape(n),
                          normal=np.asarray(nrm, np.float32).reshape(n, 3),
                          tri=np.asarray(tri, np.int32).reshape(n))
    return res


def offset_rays(L, bbox, w, r, axis, pixels, eps=1e-5):
    """The same result on chosen rays only: for each pixel of ``pixels`` on
    the ``axis``-LDNI, a list of (depth, normal, id)."""
    union = r > 0
    rr = abs(float(np.float32(r)))
    b = bbox_f32(bbox)
    centres = sphere_centres(L, bbox, w)
    a = axis
    u, v = (a + 1) % 3, (a + 2) % 3
    cu, cv = _centres(b[u], b[3 + u], w), _centres(b[v], b[3 + v], w)
    srt = np.argsort(centres[:, u], kind="stable")
    order = (srt, centres[srt, u])
    ax = L[a]
    out = []
    for p in pixels:
        p = int(p)
        o0, o1 = int(ax.offsets[p]), int(ax.offsets[p + 1])
        ev = _ray_events(a, cu[p % w], cv[p // w], centres, rr, b[a], union, order)
        out.append(offset_pixel(ax.depth[o0:o1], ax.normal[o0:o1], ax.tri[o0:o1], ev, union, eps))
    return out
