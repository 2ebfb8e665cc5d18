"""Pins of the Boolean-operation oracle (Sec. 4.1, Fig. 5; small interval
removal, Sec. 4.1.1) against what the mathematics fixes: point-membership
evaluation of the 1D sets, set identities, the paper's claim that
(A n B) - A is empty on one grid, and closed forms for sampled boxes."""
import numpy as np
import pytest

import oracle
from oracle import boolean as ob


OPS = (ob.UNION, ob.INTERSECTION, ob.DIFFERENCE)


def _brute(da, db, op, eps):
    """Boundary depths of the result by evaluating the operation between
    consecutive distinct sample depths (a formulation independent of the
    oracle's slicing)."""
    def segs(d):
        n = len(d) // 2 * 2
        return [(float(d[i]), float(d[i + 1])) for i in range(0, n, 2)]
    sa, sb = segs(da), segs(db)
    pts = sorted({z for s in sa + sb for z in s})
    if len(pts) < 2:
        return []
    def member(segs_, z):
        return any(s <= z <= e for s, e in segs_)
    def f(z):
        a, b = member(sa, z), member(sb, z)
        return {ob.UNION: a or b, ob.INTERSECTION: a and b, ob.DIFFERENCE: a and not b}[op]
    gaps = [f(0.5 * (pts[k] + pts[k + 1])) for k in range(len(pts) - 1)]
    bounds = []
    for k, z in enumerate(pts):
        left = gaps[k - 1] if k > 0 else False
        right = gaps[k] if k < len(gaps) else False
        if left != right:
            bounds.append(z)
    vols = [(bounds[i], bounds[i + 1]) for i in range(0, len(bounds), 2)]
    return [z for s, e in vols if e - s > 0 and e - s >= eps for z in (s, e)]


def _rule_ref(da, db, z, op):
    na, nb = len(da) // 2 * 2, len(db) // 2 * 2
    for i in range(na):
        if float(da[i]) == z:
            return (0, i, False)
    for j in range(nb):
        if float(db[j]) == z:
            return (1, j, op == ob.DIFFERENCE)
    raise AssertionError


def _depths(da, db, res):
    return [float(da[k]) if s == 0 else float(db[k]) for s, k, _ in res]


@pytest.mark.parametrize("seed", range(6))
def test_matches_point_membership(seed):
    rng = np.random.default_rng(seed)
    for _ in range(400):
        # small integer depths: many ties between and within the solids
        da = np.sort(rng.integers(0, 12, rng.integers(0, 9))).astype(np.float32)
        db = np.sort(rng.integers(0, 12, rng.integers(0, 9))).astype(np.float32)
        for op in OPS:
            for eps in (0.0, 1.5, 4.0):
                res = ob.boolean_pixel(da, db, op, eps)
                got = _depths(da, db, res)
                assert got == _brute(da, db, op, eps), (da, db, op, eps)
                assert res == [_rule_ref(da, db, z, op) for z in got]


def test_identities_on_random_lists():
    rng = np.random.default_rng(7)
    empty = np.zeros(0, np.float32)
    for _ in range(300):
        a = np.sort(rng.random(2 * rng.integers(0, 5))).astype(np.float32)
        b = np.sort(rng.random(2 * rng.integers(0, 5))).astype(np.float32)
        dep = lambda x, y, op: _depths(x, y, ob.boolean_pixel(x, y, op, 0.0))
        assert dep(a, empty, ob.UNION) == dep(a, a, ob.INTERSECTION) == dep(a, empty, ob.DIFFERENCE)
        assert dep(a, empty, ob.INTERSECTION) == [] and dep(a, a, ob.DIFFERENCE) == []
        assert dep(a, b, ob.UNION) == dep(b, a, ob.UNION)
        assert dep(a, b, ob.INTERSECTION) == dep(b, a, ob.INTERSECTION)
        # the difference and the intersection split A
        d, i = dep(a, b, ob.DIFFERENCE), dep(a, b, ob.INTERSECTION)
        assert dep(np.array(d, np.float32), np.array(i, np.float32), ob.INTERSECTION) == []


def _box(lo, hi):
    """Closed axis-aligned box mesh, outward winding."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x, y, z] for z in (z0, z1) for y in (y0, y1) for x in (x0, x1)], np.float32)
    f = [(0, 2, 1), (1, 2, 3), (4, 5, 6), (5, 7, 6), (0, 1, 4), (1, 5, 4),
         (2, 6, 3), (3, 6, 7), (0, 4, 2), (2, 4, 6), (1, 3, 5), (3, 7, 5)]
    return v, np.array(f, np.int32)


BBOX = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]


def _zaxis(v, f, w=16):
    return oracle.sample(v, f, BBOX, w, axes="z")[2]


def test_boxes_closed_form():
    """Along z, pixels inside both boxes' footprints see A = [-0.5, 0.25]
    and B = [-0.125, 0.625]: union [-0.5, 0.625], intersection
    [-0.125, 0.25], difference [-0.5, -0.125] ending on B's entering face
    with its normal reversed to +z."""
    A = _zaxis(*_box((-0.5, -0.5, -0.5), (0.25, 0.25, 0.25)))
    B = _zaxis(*_box((-0.125, -0.125, -0.125), (0.625, 0.625, 0.625)))
    w = 16
    both = [(j * w + i) for j in range(w) for i in range(w)
            if -0.125 < -1 + (i + 0.5) * 2 / w < 0.25 and -0.125 < -1 + (j + 0.5) * 2 / w < 0.25]
    assert both
    cases = {"union": [0.5, 1.625], "intersection": [0.875, 1.25], "difference": [0.5, 0.875]}
    for name, want in cases.items():
        r = ob.boolean(A, B, name)
        for p in both:
            s, e = int(r.offsets[p]), int(r.offsets[p + 1])
            assert list(r.depth[s:e]) == want, (name, p)
            if name == "difference":
                assert list(r.normal[e - 1]) == [0.0, 0.0, 1.0]
                assert r.tri[e - 1] < 0 and r.tri[s] >= 0


def test_tangent_boxes():
    """Boxes touching along z = 0.25: their intersection has zero
    thickness and vanishes; their union is one volume with no inner face."""
    A = _zaxis(*_box((-0.5, -0.5, -0.5), (0.5, 0.5, 0.25)))
    B = _zaxis(*_box((-0.5, -0.5, 0.25), (0.5, 0.5, 0.75)))
    assert ob.boolean(A, B, "intersection").n == 0
    u = ob.boolean(A, B, "union")
    ca = np.diff(A.offsets.astype(np.int64))
    assert (np.diff(u.offsets.astype(np.int64)) == ca).all()
    for p in np.nonzero(ca)[0]:
        s = int(u.offsets[p])
        assert list(u.depth[s:s + 2]) == [0.5, 1.75]


def test_intersection_minus_a_is_empty_on_one_grid():
    """Sec. 4.1.1: with both solids sampled on the same grid, (A n B) - A
    is empty (small interval removal at eps = 1e-5)."""
    from paper_1009_0794_amd import meshgen
    va, fa = meshgen.icosphere(2, radius=0.7)
    vb, fb = meshgen.torus(24, 12, 0.5, 0.2, center=(0.3, 0.1, 0.0))
    for axis in range(3):
        a = oracle.sample(va, fa, BBOX, 24, axes="xyz")[axis]
        b = oracle.sample(vb, fb, BBOX, 24, axes="xyz")[axis]
        inter = ob.boolean(a, b, "intersection")
        assert inter.n > 0
        assert ob.boolean(inter, a, "difference").n == 0
        # and (A u B) n A has A's volumes
        ua = ob.boolean(ob.boolean(a, b, "union"), a, "intersection")
        for p in range(24 * 24):
            got = list(ua.depth[ua.offsets[p]:ua.offsets[p + 1]])
            assert got == list(a.depth[a.offsets[p]:a.offsets[p + 1]])


def _pixel_c(da, db, op, eps):
    """One pixel through the C restatement (boolean_c) as a 1 x 1 LDNI."""
    def one(d):
        n = len(d)
        return oracle.AxisLDNI(w=1, offsets=np.array([0, n], np.uint32), depth=np.asarray(d, np.float32),
                               normal=np.tile(np.float32([0, 0, 1]), (n, 1)),
                               tri=np.arange(n, dtype=np.int32))
    r = ob.boolean_c(one(da), one(db), op, eps)
    # source of each result sample: A's ids are 0..na-1, B's become -1 - j
    return [(0, int(t), False) if t >= 0 else (1, int(-1 - t), op == ob.DIFFERENCE) for t in r.tri], r


@pytest.mark.parametrize("seed", range(6))
def test_c_oracle_matches_point_membership(seed):
    """The C restatement used for whole large images, pinned the same way as
    the Python one: result end points against point membership between
    consecutive distinct depths, and the end-point sample rule; the normal
    of an end point from B is reversed only in the difference."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(300):
        da = np.sort(rng.integers(0, 12, rng.integers(0, 9))).astype(np.float32)
        db = np.sort(rng.integers(0, 12, rng.integers(0, 9))).astype(np.float32)
        for op in OPS:
            for eps in (0.0, 1.5, 4.0):
                res, r = _pixel_c(da, db, op, eps)
                got = _depths(da, db, res)
                assert got == _brute(da, db, op, eps), (da, db, op, eps)
                assert res == [_rule_ref(da, db, z, op) for z in got]
                assert list(r.depth) == got
                for (solid, _, rev), nz in zip(res, r.normal[:, 2]):
                    assert nz == (-1.0 if rev else 1.0)
