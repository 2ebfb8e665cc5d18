"""Pins of the grid-node classification oracle (Definition 3; Sec. 5.1, step
1) against what geometry and the definition fix independently of its code:
closed forms for boxes (faces on and between nodes), the generalized winding
number of closed meshes (each LDNI's vote on its own), a node-by-node brute
force on tiny grids, and the identities of a two-of-three vote."""
import math

import numpy as np
import pytest

import oracle
from oracle import nodes as on
from paper_1009_0794_amd import meshgen as mg

BBOX = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]


def test_node_depths_closed_form():
    """On [-1, 1] with w = 16 the nodes sit at -1 + (t + 0.5)/8 exactly."""
    t = np.arange(16)
    assert np.array_equal(on.node_coordinates(-1.0, 1.0, 16), (-1 + (t + 0.5) / 8).astype(np.float32))
    assert np.array_equal(on.node_depths(-1.0, 1.0, 16), ((t + 0.5) / 8).astype(np.float32))
    # a box that does not start at zero: depths are measured from lo
    assert np.array_equal(on.node_depths(2.0, 6.0, 4), np.array([0.5, 1.5, 2.5, 3.5], np.float32))


def test_ray_rule_by_hand():
    """Nodes at depths 0.5, 1.5, ..., 7.5; G2 half-open volumes, G3 odd
    counts, ties and zero-thickness volumes."""
    d = np.arange(8, dtype=np.float32) + np.float32(0.5)
    cases = [
        ([], []),
        ([1.5, 3.5], [1, 2]),                # enter on a node: inside; leave on a node: outside
        ([1.0, 3.0], [1, 2]),                # between nodes
        ([1.5, 3.5, 3.5, 5.5], [1, 2, 3, 4]),  # touching volumes leave no gap
        ([2.5, 2.5], []),                    # zero thickness holds nothing
        ([1.5, 3.5, 4.5], [1, 2]),           # the unpaired last sample is ignored
        ([-5.0, 100.0], list(range(8))),
        ([0.0, 0.5, 7.5, 9.0], [7]),
    ]
    for samples, want in cases:
        got = np.nonzero(on.ray_inside(np.array(samples, np.float32), d))[0].tolist()
        assert got == want, (samples, got, want)


def _box_expect(lo, hi, w):
    c = [on.node_coordinates(BBOX[a], BBOX[3 + a], w).astype(np.float64) for a in range(3)]
    inside = [(lo[a] <= c[a]) & (c[a] < hi[a]) for a in range(3)]
    return inside[2][:, None, None] & inside[1][None, :, None] & inside[0][None, None, :]


@pytest.mark.parametrize("lo,hi", [
    ((-0.5625, -0.3, -0.375), (0.4, 0.4375, 0.3125)),    # faces on nodes (-0.5625, 0.4375, ...) and between
    ((-0.9375, -0.9375, -0.9375), (0.9375, 0.9375, 0.9375)),
    ((-0.31, 0.02, -0.77), (0.23, 0.61, 0.05)),
])
def test_boxes_closed_form(lo, hi):
    """Node inside iff lo <= c < hi on every axis (the sampler's tie rule
    puts rays on a lower face inside, on an upper face outside; G2 does the
    same along the ray); all three LDNIs agree."""
    w = 16
    v, f = mg.box_mesh(lo, hi)
    L = oracle.sample(v, f, BBOX, w, axes="xyz")
    inside, votes = on.classify(L[0], L[1], L[2], BBOX, w)
    want = _box_expect(np.float32(lo).astype(np.float64), np.float32(hi).astype(np.float64), w)
    assert want.any() and not want.all()
    for vote in votes:
        assert np.array_equal(vote, want)
    assert np.array_equal(inside, want)
    assert on.stats(inside, votes) == (int(want.sum()), 0)


def test_faces_through_nodes_of_an_uneven_box():
    """G1: with a box whose node coordinates are not exact binary fractions,
    box faces placed exactly on node coordinates still put the nodes of a
    lower face inside and those of an upper face outside (a sample on the
    node and the node itself get the same float32 depth)."""
    bbox = [-1.1, -0.9, -1.3, 1.2, 1.05, 0.95]
    w = 16
    b = oracle.bbox_f32(bbox)
    c = [on.node_coordinates(b[a], b[3 + a], w) for a in range(3)]
    for t0, t1 in ((3, 12), (0, 15), (5, 6)):
        lo = tuple(float(c[a][t0]) for a in range(3))
        hi = tuple(float(c[a][t1]) for a in range(3))
        v, f = mg.box_mesh(lo, hi)
        L = oracle.sample(v, f, bbox, w, axes="xyz")
        inside, votes = on.classify(L[0], L[1], L[2], bbox, w)
        want = np.zeros((w, w, w), bool)
        want[t0:t1, t0:t1, t0:t1] = True
        for vote in votes:
            assert np.array_equal(vote, want), (t0, t1)
        assert np.array_equal(inside, want)


def _winding_numbers(v, f, pts):
    """Generalized winding number of a closed outward mesh at pts (solid
    angles, Van Oosterom and Strackee), float64."""
    v = np.asarray(v, np.float64)
    f = np.asarray(f, np.int64)
    out = np.zeros(len(pts))
    for s in range(0, len(pts), 2048):
        p = pts[s:s + 2048, None, :]
        A, B, C = v[f[:, 0]][None] - p, v[f[:, 1]][None] - p, v[f[:, 2]][None] - p
        la, lb, lc = (np.linalg.norm(X, axis=2) for X in (A, B, C))
        num = np.einsum("nti,nti->nt", A, np.cross(B, C))
        den = (la * lb * lc + np.einsum("nti,nti->nt", A, B) * lc
               + np.einsum("nti,nti->nt", B, C) * la + np.einsum("nti,nti->nt", C, A) * lb)
        out[s:s + 2048] = (2.0 * np.arctan2(num, den)).sum(1) / (4.0 * math.pi)
    return out


def _solids():
    rng = np.random.default_rng(11)
    a = mg.icosphere(2, radius=0.42, center=(0.37, -0.29, 0.11))
    b = mg.torus(32, 16, 0.38, 0.15, center=(-0.38, 0.3, -0.2), rot=mg.random_rotation(rng))
    return mg.concat([a, b])


def test_each_vote_is_point_membership():
    """Away from the surface every LDNI's vote equals the winding-number
    inside test of the closed mesh (an off-centre sphere and a rotated torus,
    so a swapped frame or node index changes the answer)."""
    v, f = _solids()
    w = 24
    L = oracle.sample(v, f, BBOX, w, axes="xyz")
    inside, votes = on.classify(L[0], L[1], L[2], BBOX, w)
    c = [on.node_coordinates(BBOX[a], BBOX[3 + a], w).astype(np.float64) for a in range(3)]
    K, J, I = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    pts = np.stack([I.ravel(), J.ravel(), K.ravel()], 1)
    wn = _winding_numbers(np.asarray(v, np.float32), f, pts).reshape(w, w, w)
    clear = np.abs(wn - np.round(wn)) < 1e-6
    truth = np.round(wn) >= 1
    assert clear.mean() > 0.99 and truth[clear].mean() > 0.05
    for vote in votes:
        assert np.array_equal(vote[clear], truth[clear])
    assert np.array_equal(inside[clear], truth[clear])
    assert on.stats(inside, votes)[1] == 0


def _random_axis(rng, w, d_nodes):
    """Sorted lists mixing node depths (ties) with other values; odd counts
    and empty pixels included."""
    cnt = rng.integers(0, 7, w * w)
    cnt[rng.random(w * w) < 0.2] = 0
    off = np.zeros(w * w + 1, np.uint32)
    off[1:] = np.cumsum(cnt)
    parts = []
    for c in cnt:
        pick = np.where(rng.random(c) < 0.5, rng.choice(d_nodes, c),
                        rng.uniform(-0.5, float(d_nodes[-1]) + 0.5, c).astype(np.float32))
        parts.append(np.sort(pick.astype(np.float32)))
    n = int(off[-1])
    dep = np.concatenate(parts + [np.zeros(0, np.float32)])
    return oracle.AxisLDNI(w=w, offsets=off, depth=dep, normal=np.zeros((n, 3), np.float32),
                           tri=np.zeros(n, np.int32))


def _random_three(seed, w, bbox=BBOX):
    rng = np.random.default_rng(seed)
    b = oracle.bbox_f32(bbox)
    return [_random_axis(rng, w, on.node_depths(b[a], b[3 + a], w)) for a in range(3)]


@pytest.mark.parametrize("seed,w", [(0, 1), (1, 3), (2, 5)])
def test_brute_force_node_by_node(seed, w):
    """Node-major evaluation with plain loops: for each node, find its pixel
    on each image from the frame, count the paired samples at or before the
    node's depth, and take the majority."""
    bbox = [-1.0, -0.5, 0.25, 1.5, 2.0, 1.0]
    x, y, z = _random_three(seed, w, bbox)
    inside, _ = on.classify(x, y, z, bbox, w)
    b = oracle.bbox_f32(bbox)
    for k in range(w):
        for j in range(w):
            for i in range(w):
                node = (i, j, k)
                votes = 0
                for a, ax in enumerate((x, y, z)):
                    u, vv = (a + 1) % 3, (a + 2) % 3
                    p = node[vv] * w + node[u]
                    h = (b[3 + a] - b[a]) / w
                    c = np.float32(b[a] + (node[a] + 0.5) * h)
                    d = np.float32(float(c) - b[a])
                    s = ax.depth[int(ax.offsets[p]):int(ax.offsets[p + 1])]
                    s = s[:len(s) // 2 * 2]
                    votes += sum(1 for q in s if q <= d) % 2
                assert inside[k, j, i] == (votes >= 2), (node, votes)


def test_two_of_three_identities():
    """A vote of all-inside on one axis leaves the union of the other two, a
    vote of all-outside their intersection; two empty axes leave nothing."""
    w = 12
    x, y, z = _random_three(5, w)
    _, (vx, vy, vz) = on.classify(x, y, z, BBOX, w)
    assert (vy != vz).mean() > 0.2
    full = oracle.AxisLDNI(w=w, offsets=(2 * np.arange(w * w + 1)).astype(np.uint32),
                           depth=np.tile(np.array([-1.0, 1e30], np.float32), w * w),
                           normal=np.zeros((2 * w * w, 3), np.float32), tri=np.zeros(2 * w * w, np.int32))
    empty = oracle.AxisLDNI(w=w, offsets=np.zeros(w * w + 1, np.uint32), depth=np.zeros(0, np.float32),
                            normal=np.zeros((0, 3), np.float32), tri=np.zeros(0, np.int32))
    assert np.array_equal(on.classify(full, y, z, BBOX, w)[0], vy | vz)
    assert np.array_equal(on.classify(empty, y, z, BBOX, w)[0], vy & vz)
    assert np.array_equal(on.classify(x, full, z, BBOX, w)[0], vx | vz)
    assert np.array_equal(on.classify(x, y, empty, BBOX, w)[0], vx & vy)
    assert not on.classify(empty, empty, z, BBOX, w)[0].any()
    assert on.classify(full, full, z, BBOX, w)[0].all()


def test_unpaired_last_sample_is_ignored():
    """Appending a sample beyond every node to some pixels (odd counts)
    changes no vote."""
    w = 10
    x, y, z = _random_three(7, w)
    ref = on.classify(x, y, z, BBOX, w)
    rng = np.random.default_rng(8)
    cnt = np.diff(y.offsets.astype(np.int64))
    add = (cnt % 2 == 0) & (rng.random(w * w) < 0.5)
    parts = []
    for p in range(w * w):
        s = y.depth[y.offsets[p]:y.offsets[p + 1]]
        parts.append(np.append(s, np.float32(50.0)) if add[p] else s)
    off = np.zeros(w * w + 1, np.uint32)
    off[1:] = np.cumsum(cnt + add)
    n = int(off[-1])
    y2 = oracle.AxisLDNI(w=w, offsets=off, depth=np.concatenate(parts).astype(np.float32),
                         normal=np.zeros((n, 3), np.float32), tri=np.zeros(n, np.int32))
    got = on.classify(x, y2, z, BBOX, w)
    assert np.array_equal(got[0], ref[0])
    assert all(np.array_equal(a, b) for a, b in zip(got[1], ref[1]))


def test_classify_at_matches_dense():
    w = 9
    x, y, z = _random_three(3, w)
    inside, _ = on.classify(x, y, z, BBOX, w)
    rng = np.random.default_rng(4)
    i, j, k = rng.integers(0, w, (3, 200))
    assert np.array_equal(on.classify_at(x, y, z, BBOX, w, i, j, k), inside[k, j, i])
