"""Tiny closed meshes placed exactly on pixel-centre rays (bbox [0,8]^3,
w = 8, centres at k + 1/2), used by the exact fixtures and the parity tests."""
from __future__ import annotations

import numpy as np
from scipy.spatial import ConvexHull

from paper_1009_0794_amd import meshgen as mg

BOX8 = (0.0, 0.0, 0.0, 8.0, 8.0, 8.0)


def _oriented_hull(points):
    """Closed convex hull of lattice points, every triangle turned outward."""
    pts = np.asarray(points, dtype=np.float64)
    hull = ConvexHull(pts, qhull_options="Qt")
    used = np.unique(hull.simplices)
    remap = -np.ones(len(pts), dtype=np.int64)
    remap[used] = np.arange(len(used))
    verts = pts[used]
    c = verts.mean(0)
    tris = []
    for s in hull.simplices:
        a, b, d = (int(remap[k]) for k in s)
        n = np.cross(verts[b] - verts[a], verts[d] - verts[a])
        tris.append((a, b, d) if np.dot(n, verts[a] - c) > 0 else (a, d, b))
    return verts, np.array(tris, dtype=np.int64)


def polycube(cells, offset=0.5):
    """Boundary of a union of unit voxels (integer cells), each square face
    split into two triangles, corners at integer + offset."""
    cells = set(map(tuple, cells))
    vid, verts, tris = {}, [], []

    def V(p):
        if p not in vid:
            vid[p] = len(verts)
            verts.append(p)
        return vid[p]

    for (x, y, z) in cells:
        for axis in range(3):
            for side in (0, 1):
                nb = [x, y, z]
                nb[axis] += 1 if side else -1
                if tuple(nb) in cells:
                    continue
                u, v = (axis + 1) % 3, (axis + 2) % 3
                base = [x, y, z]
                base[axis] += side
                corners = []
                for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):
                    q = list(base)
                    q[u] += du
                    q[v] += dv
                    corners.append(V(tuple(q)))
                a, b, c, d = corners
                # (u, v, axis) is right-handed: counter-clockwise in (u,v)
                # faces +axis
                if side:
                    tris += [(a, b, c), (a, c, d)]
                else:
                    tris += [(a, c, b), (a, d, c)]
    verts = np.array(verts, dtype=np.float64) + offset
    return verts, np.array(tris, dtype=np.int64)


def _fixtures():
    out = {}
    v, f = mg.octahedron((3.5, 3.5, 3.5), 2.0)
    out["octa_on_centres"] = (v, f, BOX8, 8)
    v, f = mg.box_mesh((1.5, 2.5, 0.5), (4.5, 5.5, 6.5))
    out["box_on_centres"] = (v, f, BOX8, 8)
    cells = [(1, 1, 1), (2, 1, 1), (3, 1, 1), (1, 2, 1), (1, 3, 1), (1, 1, 2), (2, 2, 2),
             (2, 1, 2), (1, 2, 2), (4, 4, 4), (4, 5, 4), (5, 4, 4), (3, 2, 2), (3, 1, 2)]
    v, f = polycube(cells)
    out["polycube_on_centres"] = (v, f, BOX8, 8)
    rng = np.random.default_rng(11)
    pts = rng.integers(0, 8, size=(14, 3)) + 0.5
    v, f = _oriented_hull(pts)
    out["lattice_hull"] = (v, f, BOX8, 8)
    pts = rng.integers(0, 16, size=(12, 3)) * 0.5 + 0.25
    v, f = _oriented_hull(pts)
    out["half_lattice_hull"] = (v, f, BOX8, 8)
    # generic (no ties): rotated, shifted level-1 icosphere, non-cubic box
    v, f = mg.icosphere(1, 2.7, (4.1, 3.9, 4.3), mg.random_rotation(np.random.default_rng(5)))
    out["generic_ico1"] = (v, f, (0.0, 0.0, 0.0, 8.0, 7.5, 9.0), 9)
    # two octahedra with coincident silhouettes along x
    v1, f1 = mg.octahedron((2.5, 3.5, 3.5), 1.0)
    v2, f2 = mg.octahedron((5.5, 3.5, 3.5), 2.0)
    vv, ff = mg.concat([(v1, f1), (v2, f2)])
    out["two_octa"] = (vv.astype(np.float64), ff.astype(np.int64), BOX8, 8)
    return {k: (np.asarray(v, np.float32), np.asarray(f, np.int32), bb, w)
            for k, (v, f, bb, w) in out.items()}


FIXTURES = _fixtures()
