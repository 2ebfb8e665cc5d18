"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: closed forms (boxes, pixel
centres), exact rational brute force on tiny adversarial meshes, invariants
(even counts on closed meshes, Definition 4; alternating entering/leaving
normals; sortedness, Definition 1), the divergence-theorem volume measured by
the inside intervals (Sec. 2 after Proposition 1) and analytic spheres.
"""
import glob
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1009_0794_amd import meshgen as mg
from tests.meshcheck import ldni_volume, volume
from tests.golden.fixture_meshes import FIXTURES, BOX8, polycube

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def f32ulp(x):
    x = np.abs(np.float32(x))
    return float(np.spacing(x)) if x > 0 else float(np.float32(1.4e-45))


# ---------------------------------------------------------------- centres

def test_pixel_centres_closed_form():
    """bbox [0,8]^3, w=8: centres are exactly k + 1/2 on every axis
    (Sec. 3: pixels are addressed at their centres)."""
    for a in range(3):
        cu, cv = oracle.pixel_centres(BOX8, 8, a)
        assert np.array_equal(cu, np.arange(8) + 0.5)
        assert np.array_equal(cv, np.arange(8) + 0.5)


def test_pixel_centres_cyclic_frame():
    """Non-cubic box: axis x images (y,z), axis y images (z,x), axis z
    images (x,y); pitch (hi-lo)/w per image axis."""
    bb = (0.0, 0.0, 0.0, 8.0, 16.0, 32.0)
    k = np.arange(8) + 0.5
    cu, cv = oracle.pixel_centres(bb, 8, 0)
    assert np.array_equal(cu, 2 * k) and np.array_equal(cv, 4 * k)
    cu, cv = oracle.pixel_centres(bb, 8, 1)
    assert np.array_equal(cu, 4 * k) and np.array_equal(cv, k)
    cu, cv = oracle.pixel_centres(bb, 8, 2)
    assert np.array_equal(cu, k) and np.array_equal(cv, 2 * k)


def test_three_axes_share_grid_nodes():
    """Definition 3: the three images' rays meet at the nodes of one grid, so
    the centre coordinate along each world axis is the same on every image."""
    bb = (-1.1, -0.7, -2.3, 1.3, 1.9, 0.4)
    w = 97
    world = {}
    for a in range(3):
        cu, cv = oracle.pixel_centres(bb, w, a)
        for d, c in (((a + 1) % 3, cu), ((a + 2) % 3, cv)):
            if d in world:
                assert np.array_equal(world[d].view(np.uint32), c.view(np.uint32))
            world[d] = c


# ---------------------------------------------------------------- boxes

def _box_expect(lo, hi, bbox, w, axis):
    u, v = (axis + 1) % 3, (axis + 2) % 3
    cu, cv = oracle.pixel_centres(bbox, w, axis)
    iu = (cu >= np.float32(lo[u])) & (cu < np.float32(hi[u]))
    jv = (cv >= np.float32(lo[v])) & (cv < np.float32(hi[v]))
    return (jv[:, None] & iu[None, :]).ravel()


@pytest.mark.parametrize("lo,hi,bbox,w", [
    ((1.0, 3.0, 0.5), (2.5, 6.5, 7.0), BOX8, 8),
    ((1.5, 2.5, 0.5), (4.5, 5.5, 6.5), BOX8, 8),
    ((-0.3, 0.1, -0.9), (0.77, 0.55, 0.2), (-1, -1, -1, 1, 1, 1), 37),
    ((0.0, 0.0, 0.0), (8.0, 8.0, 8.0), BOX8, 8),
])
def test_box_closed_form(lo, hi, bbox, w):
    """An axis-aligned box: 2 samples where lo_u <= c_u < hi_u and
    lo_v <= c_v < hi_v, else 0; side faces are parallel to the ray and never
    hit (the note after Definition 1); depths are the two face coordinates
    minus lo_a, normals -e_a then +e_a."""
    v, f = mg.concat([mg.box_mesh(lo, hi)])
    res = oracle.sample(v, f, bbox, w)
    for a in range(3):
        r = res[a]
        inside = _box_expect(lo, hi, bbox, w, a)
        assert np.array_equal(r.counts, np.where(inside, 2, 0))
        lo_a = np.float32(bbox[a])
        d0 = np.float32(np.float64(np.float32(lo[a])) - np.float64(lo_a))
        d1 = np.float32(np.float64(np.float32(hi[a])) - np.float64(lo_a))
        assert np.array_equal(r.depth[0::2], np.full(r.n // 2, d0, np.float32))
        assert np.array_equal(r.depth[1::2], np.full(r.n // 2, d1, np.float32))
        e = np.zeros(3, np.float32)
        e[a] = 1
        assert np.array_equal(r.normal[0::2], np.tile(-e, (r.n // 2, 1)))
        assert np.array_equal(r.normal[1::2], np.tile(e, (r.n // 2, 1)))


def test_box_volume_exact():
    """Box aligned to pixel cells: the LDNI volume equals the box volume."""
    v, f = mg.concat([mg.box_mesh((1.0, 2.0, 3.0), (5.0, 7.0, 4.0))])
    res = oracle.sample(v, f, BOX8, 8)
    for a in range(3):
        assert ldni_volume(res[a], BOX8, a) == pytest.approx(4 * 5 * 1, abs=1e-9)


# ---------------------------------------------------------------- exact fixtures

def _golden_files():
    return sorted(glob.glob(os.path.join(GOLDEN, "*.json")))


@pytest.mark.parametrize("path", _golden_files(), ids=lambda p: os.path.basename(p)[:-5])
@pytest.mark.parametrize("brute", [False, True])
def test_against_exact_fixtures(path, brute):
    """Counts, hit triangles and depths against the rational evaluation of the
    definition, with rays through vertices and edges (Remark 1)."""
    doc = json.load(open(path))
    v = np.array(doc["verts"], np.float32)
    f = np.array(doc["tris"], np.int32)
    w = doc["w"]
    res = oracle.sample(v, f, doc["bbox"], w, brute=brute)
    for an, pix in doc["axes"].items():
        r = res["xyz".index(an)]
        assert np.array_equal(r.counts, [len(p) for p in pix])
        _check_layout(r)
        # where the exact depths tie (silhouette pairs), the order is by id
        for p, hits in enumerate(pix):
            s = int(r.offsets[p])
            for k in range(len(hits) - 1):
                if Fraction(hits[k][0]) == Fraction(hits[k + 1][0]):
                    assert r.tri[s + k] < r.tri[s + k + 1] and hits[k][1] < hits[k + 1][1]
        for p, hits in enumerate(pix):
            s, e = int(r.offsets[p]), int(r.offsets[p + 1])
            got = sorted(zip(r.tri[s:e].tolist(), r.depth[s:e].tolist()))
            want = sorted((t, Fraction(d)) for d, t in hits)
            assert [t for t, _ in got] == [t for t, _ in want], (an, p)
            for (t, dg), (_, dw) in zip(got, want):
                assert abs(Fraction(dg) - dw) <= Fraction(f32ulp(float(dw))) + abs(dw) * Fraction(1, 2 ** 50)


def test_exact_fixtures_are_even():
    for path in _golden_files():
        doc = json.load(open(path))
        for an, pix in doc["axes"].items():
            assert all(len(p) % 2 == 0 for p in pix), (path, an)


def test_tie_rule_half_open_square():
    """A face with edges exactly on pixel-centre lines owns the centres on
    its low-u and low-v edges only (the ray is perturbed to (+eps, +eps^2))."""
    v, f = mg.concat([mg.box_mesh((2.5, 2.5, 2.5), (5.5, 5.5, 5.5))])
    res = oracle.sample(v, f, BOX8, 8)
    c = res[2].counts.reshape(8, 8)
    expect = np.zeros((8, 8), int)
    expect[2:5, 2:5] = 2
    assert np.array_equal(c, expect)


def test_tie_rule_diagonal_owned_once():
    """A ray through the shared diagonal of a square face hits it once, not
    twice and not zero times (Remark 1, non-silhouette edge)."""
    v, f = mg.concat([mg.box_mesh((1.5, 1.5, 1.0), (5.5, 5.5, 6.0))])
    res = oracle.sample(v, f, BOX8, 8)
    c = res[2].counts.reshape(8, 8)
    # centres (k+.5, k+.5) lie on the diagonal of the z faces
    for k in range(1, 5):
        assert c[k, k] == 2
    assert res[2].n == 2 * 16


def test_exact_oracle_closed_form_box():
    """The rational micro-oracle itself agrees with the box closed form."""
    lo, hi = (1.5, 2.5, 0.5), (4.5, 5.5, 6.5)
    v, f = mg.concat([mg.box_mesh(lo, hi)])
    ex = exact.sample(v, f, BOX8, 8)
    for a in range(3):
        inside = _box_expect(lo, hi, BOX8, 8, a)
        assert [len(p) for p in ex[a]] == list(np.where(inside, 2, 0))
        for p in ex[a]:
            if p:
                assert p[0][0] == Fraction(lo[a]) and p[1][0] == Fraction(hi[a])


def test_round_f32():
    rng = np.random.default_rng(0)
    for x in np.concatenate([rng.normal(size=200) * 10.0 ** rng.integers(-40, 30, 200),
                             [1e-45, 3e-39, 0.1, 1 / 3]]):
        assert exact.round_f32(Fraction(float(x))) == Fraction(float(np.float32(x)))


# ---------------------------------------------------------------- invariants

def _check_layout(r):
    off = r.offsets.astype(np.int64)
    assert off[0] == 0 and (np.diff(off) >= 0).all() and off[-1] == r.n
    # Definition 1: ascending depths, ties by triangle id
    pix = np.repeat(np.arange(len(off) - 1), np.diff(off))
    same = pix[1:] == pix[:-1]
    d0, d1 = r.depth[:-1][same], r.depth[1:][same]
    t0, t1 = r.tri[:-1][same], r.tri[1:][same]
    assert ((d0 < d1) | ((d0 == d1) & (t0 < t1))).all()


def _check_alternating(r, axis):
    """Closed outward shells: along the ray the normals enter (n_a < 0) and
    leave (n_a > 0) alternately."""
    off = r.offsets.astype(np.int64)
    idx = np.arange(r.n) - np.repeat(off[:-1], np.diff(off))
    na = r.normal[:, axis]
    assert (na[idx % 2 == 0] < 0).all() and (na[idx % 2 == 1] > 0).all()


def test_icosphere_c1_pins():
    m = mg.c1_icosphere()
    res = oracle.sample(m.verts, m.tris, m.bbox, m.w)
    v64 = m.verts.astype(np.float64)
    a_, b_, c_ = v64[m.tris[:, 0]], v64[m.tris[:, 1]], v64[m.tris[:, 2]]
    nrm = np.cross(b_ - a_, c_ - a_)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r_in = float(np.min(np.abs(np.einsum("ij,ij->i", nrm, a_))))
    # largest angle between a face normal and its vertices' directions
    cosmax = min(float(np.min(np.einsum("ij,ij->i", nrm, x / np.linalg.norm(x, axis=1, keepdims=True))))
                 for x in (a_, b_, c_))
    vol = volume(m.verts, m.tris)
    vols = []
    for a in range(3):
        r = res[a]
        _check_layout(r)
        _check_alternating(r, a)
        cu, cv = oracle.pixel_centres(m.bbox, m.w, a)
        CU, CV = np.meshgrid(cu.astype(np.float64), cv.astype(np.float64))
        rho2 = (CU ** 2 + CV ** 2).ravel()
        cnt = r.counts
        assert set(np.unique(cnt)) <= {0, 2}
        assert (cnt[rho2 < r_in ** 2] == 2).all()
        assert (cnt[rho2 > 1 + 1e-6] == 0).all()
        # hit points lie between the inscribed and circumscribed spheres and
        # on the plane of the hit face
        pix = np.repeat(np.arange(m.w * m.w), cnt)
        P = np.zeros((r.n, 3))
        u, v = (a + 1) % 3, (a + 2) % 3
        P[:, u] = CU.ravel()[pix]
        P[:, v] = CV.ravel()[pix]
        P[:, a] = np.float64(np.float32(m.bbox[a])) + r.depth
        rad = np.linalg.norm(P, axis=1)
        assert (rad >= r_in - 1e-6).all() and (rad <= 1 + 1e-6).all()
        A = v64[m.tris[r.tri, 0]]
        resid = np.abs(np.einsum("ij,ij->i", r.normal.astype(np.float64), P - A))
        assert resid.max() <= 1e-6 * np.sqrt(3) * 2.2
        # unit normals, pointing outward within the face's angular radius
        assert np.abs(np.linalg.norm(r.normal.astype(np.float64), axis=1) - 1).max() <= 2e-7
        assert (np.einsum("ij,ij->i", r.normal.astype(np.float64), P / rad[:, None]) >= cosmax - 1e-6).all()
        vols.append(ldni_volume(r, m.bbox, a))
    # inside intervals x pixel area = the enclosed volume (Sec. 2)
    for va in vols:
        assert abs(va - vol) / vol <= 2e-3


def test_volume_error_shrinks_with_w():
    m = mg.c1_icosphere()
    vol = volume(m.verts, m.tris)
    errs = []
    for w in (64, 128, 256):
        res = oracle.sample(m.verts, m.tris, m.bbox, w, axes="z")
        errs.append(abs(ldni_volume(res[2], m.bbox, 2) - vol) / vol)
    assert errs[2] < errs[0]


def test_brute_equals_culled_c1():
    m = mg.c1_icosphere()
    r1 = oracle.sample(m.verts, m.tris, m.bbox, m.w, brute=False)
    r2 = oracle.sample(m.verts, m.tris, m.bbox, m.w, brute=True)
    for a in range(3):
        for k in ("offsets", "tri"):
            assert np.array_equal(getattr(r1[a], k), getattr(r2[a], k))
        assert np.array_equal(r1[a].depth.view(np.uint32), r2[a].depth.view(np.uint32))
        assert np.array_equal(r1[a].normal.view(np.uint32), r2[a].normal.view(np.uint32))


def test_threads_do_not_change_result():
    m = mg.c1_icosphere()
    r1 = oracle.sample(m.verts, m.tris, m.bbox, m.w, nthreads=1)
    r2 = oracle.sample(m.verts, m.tris, m.bbox, m.w, nthreads=7)
    for a in range(3):
        assert np.array_equal(r1[a].offsets, r2[a].offsets)
        assert np.array_equal(r1[a].depth.view(np.uint32), r2[a].depth.view(np.uint32))
        assert np.array_equal(r1[a].tri, r2[a].tri)


def test_random_closed_meshes_even_and_volume():
    rng = np.random.default_rng(7)
    for k in range(6):
        parts = [mg.icosphere(int(rng.integers(1, 3)), rng.uniform(0.2, 0.5),
                              rng.uniform(-0.4, 0.4, 3), mg.random_rotation(rng)) for _ in range(1)]
        parts.append(mg.torus(24, 12, 0.5, 0.15, rng.uniform(-0.2, 0.2, 3), mg.random_rotation(rng)))
        v, f = mg.concat(parts[1:])
        bb = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
        res = oracle.sample(v, f, bb, 61)
        vol = volume(v, f)
        for a in range(3):
            assert (res[a].counts % 2 == 0).all()
            _check_layout(res[a])
            assert abs(ldni_volume(res[a], bb, a) - vol) / vol < 0.05


def test_window_restricts_pixels():
    m = mg.c1_icosphere()
    full = oracle.sample(m.verts, m.tris, m.bbox, m.w, axes="y")[1]
    part = oracle.sample(m.verts, m.tris, m.bbox, m.w, axes="y", window=(10, 90, 40, 70))[1]
    c = full.counts.reshape(m.w, m.w).copy()
    mask = np.zeros_like(c, bool)
    mask[40:70, 10:90] = True
    c[~mask] = 0
    assert np.array_equal(part.counts, c.ravel())


def test_flower_pins_small():
    """A reduced flower: even counts, strictly alternating normals (a simple
    star-shaped solid), volume within the silhouette error."""
    rng = np.random.default_rng(0)
    v, f = mg.concat([mg.uv_flower(64, 128, rng)])
    bb = (-1.4, -1.4, -1.4, 1.4, 1.4, 1.4)
    res = oracle.sample(v, f, bb, 128)
    vol = volume(v, f)
    for a in range(3):
        _check_layout(res[a])
        _check_alternating(res[a], a)
        assert abs(ldni_volume(res[a], bb, a) - vol) / vol < 5e-3


# ---------------------------------------------------------------- errors

def test_oracle_rejects_bad_input():
    v, f = mg.concat([mg.box_mesh((0, 0, 0), (1, 1, 1))])
    bad = f.copy()
    bad[3, 1] = len(v)
    with pytest.raises(oracle.OracleError) as e:
        oracle.sample(v, bad, BOX8, 8)
    assert e.value.code == 2
    vn = v.copy()
    vn[2, 0] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.sample(vn, f, BOX8, 8)
    assert e.value.code == 6
    with pytest.raises(oracle.OracleError):
        oracle.sample(v, f, (0, 0, 0, 0, 8, 8), 8)


def test_empty_mesh():
    res = oracle.sample(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), BOX8, 5)
    for a in range(3):
        assert res[a].n == 0 and np.array_equal(res[a].offsets, np.zeros(26, np.uint32))


def test_faces_parallel_to_ray_never_hit():
    """The note after Definition 1: a face parallel to the ray is no hit, also
    when the ray runs inside it or it projects onto a single pixel centre."""
    v = np.array([[3.5, 3.5, 1.0], [3.5, 3.5, 2.0], [3.5, 3.5, 3.0],      # a point in z
                  [2.5, 4.5, 1.0], [5.5, 4.5, 1.0], [4.5, 4.5, 6.0],      # a segment in z
                  [1.0, 1.0, 1.0], [1.0, 1.0, 1.0], [1.0, 1.0, 1.0]],     # a point in 3D
                 np.float32)
    f = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]], np.int32)
    for brute in (False, True):
        res = oracle.sample(v, f, BOX8, 8, axes="z", brute=brute)
        assert res[2].n == 0
    ex = exact.sample(v, f, BOX8, 8, axes="z")
    assert sum(len(p) for p in ex[2]) == 0
