"""Pins of the offsetting oracle (Sec. 4.2; Boolean operations Sec. 4.1 with
small interval removal Sec. 4.1.1) against what geometry fixes: a
point-membership evaluation (inside H, or closer than r to some sample)
between consecutive event depths of every ray, closed forms on a sample's own
ray, the sample points behind the ids, and where each result sample lies."""
import math

import numpy as np
import pytest

import oracle
from oracle import offset as oo
from paper_1009_0794_amd import meshgen as mg

BBOX = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]


def _solid(w):
    rng = np.random.default_rng(5)
    a = mg.icosphere(2, radius=0.45, center=(0.21, -0.13, 0.07))
    b = mg.torus(16, 8, 0.4, 0.16, center=(-0.3, 0.28, -0.2), rot=mg.random_rotation(rng))
    v, f = mg.concat([a, b])
    return oracle.sample(v, f, BBOX, w, axes="xyz")


def _points(L, w):
    """Sample points in OF4 order, recomputed with plain loops."""
    b = oracle.bbox_f32(BBOX)
    pts = []
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        for p in range(w * w):
            iu, iv = p % w, p // w
            for q in range(int(L[a].offsets[p]), int(L[a].offsets[p + 1])):
                x = [0.0, 0.0, 0.0]
                x[a] = b[a] + float(L[a].depth[q])
                x[u] = float(np.float32(b[u] + (iu + 0.5) * (b[3 + u] - b[u]) / w))
                x[v] = float(np.float32(b[v] + (iv + 0.5) * (b[3 + v] - b[v]) / w))
                pts.append(x)
    return np.array(pts)


def _in_h(depths, z):
    d = np.asarray(depths, np.float64)[: len(depths) // 2 * 2]
    return any(d[k] < z < d[k + 1] for k in range(0, len(d), 2))


@pytest.mark.parametrize("w,r", [(10, 0.23), (10, -0.23), (12, 0.31), (12, -0.17)])
def test_membership_between_events(w, r):
    """Between consecutive distinct event depths of every ray, the result is
    inside exactly when the midpoint is inside H and/or within |r| of a
    sample point (union / difference); every kept volume is at least eps
    thick."""
    L = _solid(w)
    res = oo.offset(L, BBOX, w, r)
    pts = _points(L, w)
    b = oracle.bbox_f32(BBOX)
    rr = abs(float(np.float32(r)))
    checked = 0
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        for p in range(w * w):
            cu = float(np.float32(b[u] + (p % w + 0.5) * (b[3 + u] - b[u]) / w))
            cv = float(np.float32(b[v] + (p // w + 0.5) * (b[3 + v] - b[v]) / w))
            hd = L[a].depth[L[a].offsets[p]:L[a].offsets[p + 1]]
            rd = res[a].depth[res[a].offsets[p]:res[a].offsets[p + 1]]
            assert len(rd) % 2 == 0
            assert np.all(np.diff(rd.astype(np.float64)) >= 0)
            # event depths: H's samples and every sphere's chord ends on this ray
            rho2 = (cu - pts[:, u]) ** 2 + (cv - pts[:, v]) ** 2
            near = rho2 < rr * rr
            t = np.sqrt(rr * rr - rho2[near])
            ev = np.concatenate([hd.astype(np.float64),
                                 np.float32(pts[near, a] - t - b[a]).astype(np.float64),
                                 np.float32(pts[near, a] + t - b[a]).astype(np.float64)])
            ev = np.unique(ev)
            for k in range(len(ev) - 1):
                if ev[k + 1] - ev[k] < 1e-4:
                    continue  # slivers: removed by eps, checked below
                z = 0.5 * (ev[k] + ev[k + 1])
                dist2 = (cu - pts[:, u]) ** 2 + (cv - pts[:, v]) ** 2 + (b[a] + z - pts[:, a]) ** 2
                in_s = bool((dist2 < rr * rr).any())
                want = (_in_h(hd, z) or in_s) if r > 0 else (_in_h(hd, z) and not in_s)
                got = _in_h(rd, z)
                assert got == want, (a, p, z)
                checked += 1
            thick = rd[1::2].astype(np.float64) - rd[0::2].astype(np.float64)
            assert np.all(thick >= 1e-5)
    assert checked > 1000


def test_sample_ray_closed_form():
    """On a sample's own ray its sphere is hit at rho = 0, so a solid slab
    [d0, d1] along the ray becomes [d0 - r, d1 + r] (union) and, for the
    difference, loses [d0, d0 + r] and [d1 - r, d1]."""
    w = 8
    off = np.zeros(w * w + 1, np.uint32)
    p0 = 3 * w + 5
    off[p0 + 1:] = 2
    d = np.array([0.5, 1.25], np.float32)
    nrm = np.array([[-1, 0, 0], [1, 0, 0]], np.float32)
    x = oracle.AxisLDNI(w=w, offsets=off, depth=d, normal=nrm, tri=np.array([7, 8], np.int32))
    e = oracle.AxisLDNI(w=w, offsets=np.zeros(w * w + 1, np.uint32), depth=np.zeros(0, np.float32),
                        normal=np.zeros((0, 3), np.float32), tri=np.zeros(0, np.int32))
    for r in (0.125, 0.25):
        u = oo.offset({0: x, 1: e, 2: e}, BBOX, w, r)[0]
        s = slice(int(u.offsets[p0]), int(u.offsets[p0 + 1]))
        assert list(u.depth[s]) == [0.5 - r, 1.25 + r]
        assert list(u.tri[s]) == [-1, -2]            # the spheres of samples g = 0 and 1
        assert u.normal[s].tolist() == [[-1, 0, 0], [1, 0, 0]]
        dd = oo.offset({0: x, 1: e, 2: e}, BBOX, w, -r)[0]
        s = slice(int(dd.offsets[p0]), int(dd.offsets[p0 + 1]))
        assert list(dd.depth[s]) == [0.5 + r, 1.25 - r]
        assert list(dd.tri[s]) == [-1, -2]
        assert dd.normal[s].tolist() == [[-1, 0, 0], [1, 0, 0]]  # reversed sphere normals face out of H - S
        # the neighbouring ray one pixel away (h = 0.25) along y: chords of half-width sqrt(r^2 - h^2)
        q = p0 + 1
        t = math.sqrt(max(r * r - 0.0625, 0.0))
        s = slice(int(u.offsets[q]), int(u.offsets[q + 1]))
        if t > 0:
            assert list(u.depth[s]) == [np.float32(0.5 - t), np.float32(1.25 + t)] or \
                   list(u.depth[s]) == [np.float32(0.5 - t), np.float32(0.5 + t),
                                        np.float32(1.25 - t), np.float32(1.25 + t)]
        else:
            assert s.stop == s.start  # a tangent ray is not hit


@pytest.mark.parametrize("r", [0.27, -0.11])
def test_result_samples_lie_where_they_claim(r):
    """An id >= 0 is a copy of H's sample; an id -1 - g lies on the sphere of
    sample g (|x - p_g| = |r| up to the float32 depth), with the sphere's
    radial normal (reversed for the difference), and no sample of H and no
    earlier sphere has an event at that depth."""
    w = 10
    L = _solid(w)
    res = oo.offset(L, BBOX, w, r)
    pts = _points(L, w)
    b = oracle.bbox_f32(BBOX)
    rr = abs(float(np.float32(r)))
    n_sphere = 0
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        for p in range(w * w):
            cu = float(np.float32(b[u] + (p % w + 0.5) * (b[3 + u] - b[u]) / w))
            cv = float(np.float32(b[v] + (p // w + 0.5) * (b[3 + v] - b[v]) / w))
            hs = slice(int(L[a].offsets[p]), int(L[a].offsets[p + 1]))
            for q in range(int(res[a].offsets[p]), int(res[a].offsets[p + 1])):
                d, t, nrm = res[a].depth[q], int(res[a].tri[q]), res[a].normal[q]
                if t >= 0:
                    k = np.nonzero((L[a].tri[hs] == t) & (L[a].depth[hs] == d))[0]
                    assert k.size >= 1
                    assert np.array_equal(L[a].normal[hs][k[0]], nrm)
                    continue
                n_sphere += 1
                g = -1 - t
                assert d not in set(L[a].depth[hs][: (hs.stop - hs.start) // 2 * 2].tolist())
                x = np.zeros(3)
                x[a], x[u], x[v] = b[a] + float(d), cu, cv
                assert abs(np.linalg.norm(x - pts[g]) - rr) < 1e-5
                radial = (x - pts[g]) / rr * (1 if r > 0 else -1)
                assert np.allclose(nrm, radial, atol=1e-5)
                # no earlier sphere (smaller g) has an event at this depth
                rho2 = (cu - pts[:g, u]) ** 2 + (cv - pts[:g, v]) ** 2
                near = np.nonzero(rho2 < rr * rr)[0]
                tt = np.sqrt(rr * rr - rho2[near])
                ends = set(np.float32(pts[near, a] - tt - b[a]).tolist()) | \
                       set(np.float32(pts[near, a] + tt - b[a]).tolist())
                assert float(d) not in ends
    assert n_sphere > 50


def test_sphere_numbering_follows_the_samples():
    w = 6
    L = _solid(w)
    assert np.array_equal(oo.sphere_centres(L, BBOX, w), _points(L, w))


def test_tiny_radius_keeps_the_solid():
    """A radius far below the pixel size: each volume of H grows by r at both
    ends (its samples' spheres are hit on their own rays at rho = 0), and by
    less than 3r where a sample of another axis lies within r of the ray;
    any other volume is a lone sphere chord at most 2r thick."""
    w = 10
    L = _solid(w)
    r = 1e-3
    res = oo.offset(L, BBOX, w, r)
    lone = 0
    for a in range(3):
        for p in range(w * w):
            hd = L[a].depth[L[a].offsets[p]:L[a].offsets[p + 1]].astype(np.float64)
            rd = res[a].depth[res[a].offsets[p]:res[a].offsets[p + 1]].astype(np.float64)
            hv = list(zip(hd[0::2], hd[1::2]))
            for s0, s1 in zip(rd[0::2], rd[1::2]):
                inner = [(h0, h1) for h0, h1 in hv if s0 <= h0 and h1 <= s1]
                if inner:
                    # grown by r, or a little more where a nearby chord overlaps the end
                    assert inner[0][0] - 3 * r <= s0 <= inner[0][0] - r + 1e-6
                    assert inner[-1][1] + r - 1e-6 <= s1 <= inner[-1][1] + 3 * r
                else:
                    assert s1 - s0 <= 2 * r + 1e-6
                    lone += 1
            for h0, h1 in hv:
                assert any(s0 <= h0 and h1 <= s1 for s0, s1 in zip(rd[0::2], rd[1::2]))
    assert lone < 0.05 * sum(int(L[a].n) for a in range(3))


def test_pixel_rules_by_hand():
    """OF3 on hand-made events: H's samples win ties, then the sphere of the
    smaller generating sample, a sphere's enter before its exit; touching
    volumes merge; volumes thinner than eps go, one exactly eps thick stays."""
    n = lambda *v: np.array(v, np.float32)
    hd, hn, ht = np.array([1.0, 2.0], np.float32), np.array([[0, 0, -1], [0, 0, 1]], np.float32), [10, 11]
    ev = [(np.float32(1.0), 5, 0, n(1, 0, 0)), (np.float32(1.5), 5, 1, n(0, 1, 0)),
          (np.float32(2.0), 3, 0, n(0, 0, 1)), (np.float32(3.0), 3, 1, n(1, 1, 0)),
          (np.float32(3.0), 1, 0, n(0, 1, 1)), (np.float32(4.0), 1, 1, n(1, 0, 1))]
    got = oo.offset_pixel(hd, hn, ht, ev, True, 1e-5)
    # union: [1, 4]; the start at 1 is H's sample (not sphere 5), the end at 4 sphere 1's exit;
    # H's exit at 2 meets sphere 3's enter at 2, sphere 3's exit at 3 meets sphere 1's enter: no gap
    assert [(float(d), t) for d, _, t in got] == [(1.0, 10), (4.0, -2)]
    got = oo.offset_pixel(hd, hn, ht, ev, False, 1e-5)
    # difference: H = [1, 2] minus [1, 1.5]: [1.5, 2] from sphere 5's exit and H's exit
    assert [(float(d), t) for d, _, t in got] == [(1.5, -6), (2.0, 11)]
    # two spheres entering at one depth: the smaller generating sample supplies the end point
    ev2 = [(np.float32(0.5), 9, 0, n(1, 0, 0)), (np.float32(0.75), 9, 1, n(1, 0, 0)),
           (np.float32(0.5), 4, 0, n(0, 1, 0)), (np.float32(0.6), 4, 1, n(0, 1, 0))]
    got = oo.offset_pixel(np.zeros(0, np.float32), np.zeros((0, 3), np.float32), [], ev2, True, 1e-5)
    assert [(float(d), t) for d, _, t in got] == [(0.5, -5), (0.75, -10)]
    # a volume thinner than eps is removed; an unpaired last H sample is ignored
    ev3 = [(np.float32(5.0), 0, 0, n(1, 0, 0)), (np.float32(5.000001), 0, 1, n(1, 0, 0)),
           (np.float32(8.0), 1, 0, n(1, 0, 0)), (np.float32(9.0), 1, 1, n(1, 0, 0))]
    got = oo.offset_pixel(n(1.0, 2.0, 7.0), np.zeros((3, 3), np.float32), [1, 2, 3], ev3, True, 1e-5)
    assert [(float(d), t) for d, _, t in got] == [(1.0, 1), (2.0, 2), (8.0, -2), (9.0, -2)]
    # a volume exactly eps thick stays (Sec. 4.1.1 removes only thinner ones)
    got = oo.offset_pixel(n(0.5, 0.75), np.zeros((2, 3), np.float32), [1, 2], [], True, 0.25)
    assert [(float(d), t) for d, _, t in got] == [(0.5, 1), (0.75, 2)]
    # a sphere whose chord rounds to one depth enters before it exits: in a
    # group where sphere 1 also enters, the end point is sphere 0's enter
    ev4 = [(np.float32(1.0), 0, 1, n(0, 0, 1)), (np.float32(1.0), 0, 0, n(0, 0, -1)),
           (np.float32(1.0), 1, 0, n(1, 0, 0)), (np.float32(2.0), 1, 1, n(0, 1, 0))]
    got = oo.offset_pixel(np.zeros(0, np.float32), np.zeros((0, 3), np.float32), [], ev4, True, 1e-5)
    assert [(float(d), tuple(float(c) for c in nr), t) for d, nr, t in got] == \
        [(1.0, (0.0, 0.0, -1.0), -1), (2.0, (0.0, 1.0, 0.0), -2)]


def test_tangent_sphere_is_no_event():
    """A sphere exactly tangent to a ray (rho = r) does not hit it: where a
    tangent sphere of an earlier sample touches the ray at the depth at which
    a later sample's sphere enters, the end point is the later sphere's."""
    w = 8  # centres -0.875 + 0.25 i: pixels (3, 4) and (4, 4) of the z-LDNI are 0.25 apart
    off = np.zeros(w * w + 1, np.uint32)
    off[36:] = 2
    off[37:] = 4
    d = np.array([0.5, 1.0, 0.75, 1.25], np.float32)
    z = oracle.AxisLDNI(w=w, offsets=off, depth=d, normal=np.zeros((4, 3), np.float32),
                        tri=np.array([1, 2, 3, 4], np.int32))
    e = oracle.AxisLDNI(w=w, offsets=np.zeros(w * w + 1, np.uint32), depth=np.zeros(0, np.float32),
                        normal=np.zeros((0, 3), np.float32), tri=np.zeros(0, np.int32))
    res = oo.offset({0: e, 1: e, 2: z}, BBOX, w, 0.25)[2]
    s = slice(int(res.offsets[36]), int(res.offsets[37]))
    # ray (4, 4): its samples 0.75 and 1.25 (g = 2, 3) grow to [0.5, 1.5]; the spheres of
    # g = 0, 1 at pixel (3, 4) are tangent to it at depths 0.5 and 1.0
    assert [(float(x), int(t)) for x, t in zip(res.depth[s], res.tri[s])] == [(0.5, -3), (1.5, -4)]


def test_offset_rays_matches_full():
    w = 10
    L = _solid(w)
    full = oo.offset(L, BBOX, w, 0.21)
    pix = [0, 17, 45, 46, 99]
    for a in range(3):
        got = oo.offset_rays(L, BBOX, w, 0.21, a, pix)
        for p, res in zip(pix, got):
            s = slice(int(full[a].offsets[p]), int(full[a].offsets[p + 1]))
            assert [float(d) for d, _, _ in res] == full[a].depth[s].tolist()
            assert [t for _, _, t in res] == full[a].tri[s].tolist()
