"""Parity of the HIP offsetting (Sec. 4.2; Boolean operations Sec. 4.1 with
small interval removal Sec. 4.1.1) with the CPU oracle: kept samples of the
solid are copies and sphere samples are computed by the same float64
arithmetic, so offsets, depths, normals and ids must match bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from oracle import offset as oo
import paper_1009_0794_amd as ldni
from paper_1009_0794_amd import meshgen as mg
from paper_1009_0794_amd._lib import LDNIError

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BBOX = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]


def _to_gpu(axis, a: oracle.AxisLDNI) -> ldni.LDNI:
    cnt = np.diff(a.offsets.astype(np.int64))
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    return ldni.LDNI(axis, a.w, int(cnt.max()) if cnt.size else 0, t(a.offsets.view(np.int32)),
                     t(a.depth.astype(np.float32)), t(a.normal.astype(np.float32).reshape(-1, 3)),
                     t(a.tri.astype(np.int32)))


def _same(got: ldni.LDNI, ref: oracle.AxisLDNI, label):
    off = got.offsets.cpu().numpy().view(np.uint32)
    assert np.array_equal(off, ref.offsets), f"{label}: offsets ({int((off != ref.offsets).sum())} differ)"
    assert np.array_equal(got.depth.cpu().numpy().view(np.uint32), ref.depth.view(np.uint32)), f"{label}: depth"
    assert np.array_equal(got.normal.cpu().numpy().view(np.uint32).reshape(-1, 3),
                          ref.normal.view(np.uint32).reshape(-1, 3)), f"{label}: normal"
    assert np.array_equal(got.tri.cpu().numpy(), ref.tri), f"{label}: tri"
    cnt = np.diff(off.astype(np.int64))
    assert got.max_layers == (int(cnt.max()) if cnt.size else 0), f"{label}: max layers"


def _solid(w, bbox=BBOX):
    rng = np.random.default_rng(5)
    a = mg.icosphere(2, radius=0.45, center=(0.21, -0.13, 0.07))
    b = mg.torus(16, 8, 0.4, 0.16, center=(-0.3, 0.28, -0.2), rot=mg.random_rotation(rng))
    v, f = mg.concat([a, b])
    return v, f, oracle.sample(v, f, bbox, w, axes="xyz")


@pytest.mark.parametrize("w,r", [(16, 0.11), (16, -0.07), (24, 0.2), (24, -0.13), (31, 0.05)])
def test_solids_match_oracle(w, r):
    """An icosphere and a rotated torus: outer and inner offsets from below a
    pixel to several pixels, on a grid that leaves a ragged 8 x 8 tile."""
    _, _, L = _solid(w)
    ref = oo.offset(L, BBOX, w, r)
    got = ldni.offset({a: _to_gpu(a, L[a]) for a in range(3)}, BBOX, r)
    for a in range(3):
        _same(got[a], ref[a], f"w={w} r={r} axis {a}")


def test_library_sampling_end_to_end():
    """The library's own sampling followed by its offset equals the oracle's
    sampling followed by the oracle's offset."""
    w = 20
    v, f, L = _solid(w)
    vt = torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(DEV)
    ft = torch.from_numpy(np.ascontiguousarray(f, np.int32)).to(DEV)
    S = ldni.sample(vt, ft, BBOX, w, "xyz")
    got = ldni.offset(S, BBOX, 0.15)
    ref = oo.offset(L, BBOX, w, 0.15)
    for a in range(3):
        _same(got[a], ref[a], f"axis {a}")


def _random_axis(rng, w, n_max=7):
    """Sorted lists with ties and odd counts (not a solid: the operation is
    per ray, so any sorted lists are valid input)."""
    cnt = rng.integers(0, n_max, w * w)
    cnt[rng.random(w * w) < 0.3] = 0
    off = np.zeros(w * w + 1, np.uint32)
    off[1:] = np.cumsum(cnt)
    dep = np.concatenate([np.sort(rng.integers(0, 16, c)).astype(np.float32) * np.float32(0.125)
                          for c in cnt] + [np.zeros(0, np.float32)])
    n = int(off[-1])
    nrm = rng.normal(size=(n, 3)).astype(np.float32)
    return oracle.AxisLDNI(w=w, offsets=off, depth=dep, normal=nrm,
                           tri=rng.integers(0, 1 << 30, n).astype(np.int32))


@pytest.mark.parametrize("seed,w,r,eps", [(0, 1, 0.3, 1e-5), (1, 9, 0.25, 1e-5), (2, 12, -0.2, 1e-5),
                                          (3, 12, 0.125, 1e-5), (4, 12, -0.125, 0.25), (5, 9, 0.25, 0.125)])
def test_random_lists_match_oracle(seed, w, r, eps):
    """Ties between samples and chord ends on a dyadic grid (r = 1/8 and 1/4
    put chord ends on sample depths), odd counts, empty pixels; eps on the
    same grid, so volumes exactly eps thick (kept) and thinner ones meet."""
    rng = np.random.default_rng(seed)
    L = {a: _random_axis(rng, w) for a in range(3)}
    ref = oo.offset(L, BBOX, w, r, eps)
    got = ldni.offset({a: _to_gpu(a, L[a]) for a in range(3)}, BBOX, r, eps)
    for a in range(3):
        _same(got[a], ref[a], f"seed {seed} axis {a}")


@pytest.mark.parametrize("w,r_pix", [(128, 2.5), (128, 2.0), (256, 2.0)])
def test_flower_sampled_rays(w, r_pix):
    """C2's flower mesh sampled at w = 128 (the paper's offsetting
    resolution) and 256, offset out and in by 2.5 and 2 pixels (2 pixels at
    both sizes is the timed workload): 600 random rays of each axis against
    the oracle."""
    m = mg.c2_flower()
    L = oracle.sample(m.verts, m.tris, m.bbox, w, axes="xyz")
    G = {a: _to_gpu(a, L[a]) for a in range(3)}
    h = (m.bbox[3] - m.bbox[0]) / w
    rng = np.random.default_rng(2)
    for r in (r_pix * h, -r_pix * h):
        got = ldni.offset(G, m.bbox, r)
        for a in range(3):
            off = got[a].offsets.cpu().numpy().view(np.uint32).astype(np.int64)
            dep = got[a].depth.cpu().numpy()
            tri = got[a].tri.cpu().numpy()
            nrm = got[a].normal.cpu().numpy()
            pix = rng.integers(0, w * w, 600)
            ref = oo.offset_rays(L, m.bbox, w, r, a, pix)
            for p, res in zip(pix, ref):
                s = slice(off[p], off[p + 1])
                assert dep[s].view(np.uint32).tolist() == [np.float32(d).view(np.uint32) for d, _, _ in res]
                assert tri[s].tolist() == [t for _, _, t in res]
                assert np.array_equal(nrm[s].view(np.uint32),
                                      np.array([n for _, n, _ in res], np.float32).reshape(-1, 3).view(np.uint32))


@pytest.mark.parametrize("keep", [None, 32, 16, 0])
def test_kept_end_points_do_not_change_results(keep, monkeypatch):
    """The count pass keeps up to 64 end points per ray (as many as fit its
    buffer budget) and the write pass expands those rays from them, sweeping
    only the others again; every budget (64, 32, 16 or none kept) gives the
    same offsets as the oracle on sampled rays of the flower at w = 128."""
    w = 128
    if keep is not None:
        monkeypatch.setenv("LDNI_OFFSET_KEEP_BYTES", str(8 * keep * 3 * w * w))
    m = mg.c2_flower()
    L = oracle.sample(m.verts, m.tris, m.bbox, w, axes="xyz")
    G = {a: _to_gpu(a, L[a]) for a in range(3)}
    h = (m.bbox[3] - m.bbox[0]) / w
    rng = np.random.default_rng(5)
    for r in (2.0 * h, -2.0 * h):
        got = ldni.offset(G, m.bbox, r)
        for a in range(3):
            off = got[a].offsets.cpu().numpy().view(np.uint32).astype(np.int64)
            dep = got[a].depth.cpu().numpy()
            tri = got[a].tri.cpu().numpy()
            cnt = np.diff(off)
            # rays with many end points first: they take the kept or the swept path by budget
            pix = np.concatenate([np.argsort(-cnt)[:100], rng.integers(0, w * w, 200)])
            ref = oo.offset_rays(L, m.bbox, w, r, a, pix)
            for p, res in zip(pix, ref):
                s = slice(off[p], off[p + 1])
                assert dep[s].view(np.uint32).tolist() == [np.float32(d).view(np.uint32) for d, _, _ in res]
                assert tri[s].tolist() == [t for _, _, t in res]


def test_empty_solid():
    w = 9
    e = oracle.AxisLDNI(w=w, offsets=np.zeros(w * w + 1, np.uint32), depth=np.zeros(0, np.float32),
                        normal=np.zeros((0, 3), np.float32), tri=np.zeros(0, np.int32))
    got = ldni.offset({a: _to_gpu(a, e) for a in range(3)}, BBOX, 0.3)
    for a in range(3):
        assert got[a].depth.numel() == 0 and not got[a].offsets.any()


@pytest.mark.parametrize("w,r", [(20, 0.8), (24, -0.7)])
def test_large_radius_in_depth_windows(w, r):
    """A radius of many pixels: the densest rays meet 1,436 (w = 20) and
    2,082 (w = 24) events, more than one LDS window holds (1,024), and are
    swept window by window; the result matches the oracle bit for bit."""
    _, _, L = _solid(w)
    centres = oo.sphere_centres(L, BBOX, w)
    b = oracle.bbox_f32(BBOX)
    most = 0
    for a in range(3):
        u, v = (a + 1) % 3, (a + 2) % 3
        cu = ((b[u] + (np.arange(w) + 0.5) * (b[3 + u] - b[u]) / w).astype(np.float32)).astype(np.float64)
        cv = ((b[v] + (np.arange(w) + 0.5) * (b[3 + v] - b[v]) / w).astype(np.float32)).astype(np.float64)
        for p in range(w * w):
            rho2 = (cu[p % w] - centres[:, u]) ** 2 + (cv[p // w] - centres[:, v]) ** 2
            most = max(most, 2 * int((rho2 < r * r).sum()))
    assert most > 1024
    ref = oo.offset(L, BBOX, w, r)
    got = ldni.offset({a: _to_gpu(a, L[a]) for a in range(3)}, BBOX, r)
    for a in range(3):
        _same(got[a], ref[a], f"axis {a}")


def _one_ray_solid(w, depths, pixel=5):
    """x-axis LDNI with the given depths on one ray, y and z empty."""
    n = len(depths)
    off = np.zeros(w * w + 1, np.uint32)
    off[pixel + 1:] = n
    x = oracle.AxisLDNI(w=w, offsets=off, depth=np.asarray(depths, np.float32),
                        normal=np.zeros((n, 3), np.float32), tri=np.arange(n, dtype=np.int32))
    e = oracle.AxisLDNI(w=w, offsets=np.zeros(w * w + 1, np.uint32), depth=np.zeros(0, np.float32),
                        normal=np.zeros((0, 3), np.float32), tri=np.zeros(0, np.int32))
    return {0: x, 1: e, 2: e}


@pytest.mark.parametrize("volumes", [300, 700])
def test_rays_with_many_end_points(volumes):
    """A ray whose result has 600 and 1,400 end points before small volumes
    are removed (that many separate volumes of the solid and a tiny radius),
    more than one batch of 512: the end points go to the small volume
    removal in batches and the result matches the oracle."""
    w = 4
    d = np.concatenate([[0.002 * k, 0.002 * k + 0.001] for k in range(volumes)]).astype(np.float32)
    L = _one_ray_solid(w, d)
    ref = oo.offset(L, BBOX, w, 1e-5)
    assert int(np.diff(ref[0].offsets.astype(np.int64)).max()) == 2 * volumes
    got = ldni.offset({a: _to_gpu(a, L[a]) for a in range(3)}, BBOX, 1e-5)
    for a in range(3):
        _same(got[a], ref[a], f"{volumes} volumes, axis {a}")


@pytest.mark.parametrize("r", [1e-5, -1e-5, 0.3])
def test_group_of_equal_depth_larger_than_a_window(r):
    """1,200 samples of the solid at one float32 depth on one ray, with
    volumes before and after it: the group fills a whole window (1,024
    events) and is taken whole; the result matches the oracle."""
    w = 4
    d = ([0.001 * k for k in range(40)] + [0.5] * 1200 + [0.6 + 0.001 * k for k in range(40)])
    L = _one_ray_solid(w, d)
    ref = oo.offset(L, BBOX, w, r)
    got = ldni.offset({a: _to_gpu(a, L[a]) for a in range(3)}, BBOX, r)
    for a in range(3):
        _same(got[a], ref[a], f"r={r} axis {a}")


def test_bad_offsets_rejected():
    w = 8
    _, _, L = _solid(w)
    G = {a: _to_gpu(a, L[a]) for a in range(3)}
    bad = ldni.LDNI(1, w, G[1].max_layers, G[1].offsets.clone(), G[1].depth, G[1].normal, G[1].tri)
    bad.offsets[20] = bad.offsets[21] + 3
    with pytest.raises(LDNIError) as e:
        ldni.offset({0: G[0], 1: bad, 2: G[2]}, BBOX, 0.1)
    assert e.value.code == 1


def test_binning_tables_overflow():
    """A small sphere offset by a radius three times its own: the 256
    spheres of a binning workgroup hit more rays than its LDS table holds
    (1,024 slots), so some rays are counted and placed through the global
    fallback (in both binning passes) while the others go through the
    table; the result matches the oracle bit for bit."""
    w, r = 64, 0.6
    v, f = mg.icosphere(1, radius=0.2, center=(0.05, -0.03, 0.02))
    L = oracle.sample(v, f, BBOX, w, axes="xyz")
    centres = oo.sphere_centres(L, BBOX, w)
    assert len(centres) >= 256
    b = oracle.bbox_f32(BBOX)
    # the rays of image 0 that the first workgroup's 256 spheres hit
    cu = ((b[1] + (np.arange(w) + 0.5) * (b[4] - b[1]) / w).astype(np.float32)).astype(np.float64)
    cv = ((b[2] + (np.arange(w) + 0.5) * (b[5] - b[2]) / w).astype(np.float32)).astype(np.float64)
    c = centres[:256]
    d2 = (cu[None, None, :] - c[:, 1, None, None]) ** 2 + (cv[None, :, None] - c[:, 2, None, None]) ** 2
    assert int((d2 < r * r).any(axis=0).sum()) > 1024
    ref = oo.offset(L, BBOX, w, r)
    got = ldni.offset({a: _to_gpu(a, L[a]) for a in range(3)}, BBOX, r)
    for a in range(3):
        _same(got[a], ref[a], f"axis {a}")
