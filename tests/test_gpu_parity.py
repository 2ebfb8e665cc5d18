"""Parity of the HIP sampler with the CPU oracle, element by element.

Counts, offsets, triangle ids and their order must be identical; depths must
agree within 1e-5 x the box diagonal and normals within 1e-5 (float32), and
are expected to be bit-identical because both sides evaluate the same
float64 formulas in the same order.
"""
import json
import glob
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1009_0794_amd as ldni
from paper_1009_0794_amd import meshgen as mg
from tests.golden.fixture_meshes import FIXTURES, BOX8

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _diag(bbox):
    b = np.asarray(bbox, np.float64)
    return float(np.linalg.norm(b[3:] - b[:3]))


def _run(v, f, bbox, w, axes="xyz"):
    vt = torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(DEV)
    ft = torch.from_numpy(np.ascontiguousarray(f, np.int32)).to(DEV)
    out = ldni.sample(vt, ft, bbox, w, axes)
    torch.cuda.synchronize()
    return out


def _np(g):
    return (g.offsets.cpu().numpy().view(np.uint32), g.depth.cpu().numpy(),
            g.normal.cpu().numpy(), g.tri.cpu().numpy())


def compare(got, ref, bbox, bitwise=True, label=""):
    tol_d = 1e-5 * _diag(bbox)
    for a, r in ref.items():
        off, dep, nrm, tri = _np(got[a])
        assert np.array_equal(off, r.offsets), f"{label} axis {a}: offsets differ"
        assert np.array_equal(tri, r.tri), f"{label} axis {a}: triangle ids/order differ"
        if r.n:
            assert np.abs(dep.astype(np.float64) - r.depth).max() <= tol_d, f"{label} axis {a}: depth"
            assert np.abs(nrm.astype(np.float64) - r.normal).max() <= 1e-5, f"{label} axis {a}: normal"
        if bitwise:
            assert np.array_equal(dep.view(np.uint32), r.depth.view(np.uint32)), f"{label} axis {a}: depth bits"
            assert np.array_equal(nrm.view(np.uint32), r.normal.view(np.uint32)), f"{label} axis {a}: normal bits"
        cnt = np.diff(off.astype(np.int64))
        assert got[a].max_layers == (int(cnt.max()) if cnt.size else 0)


@pytest.fixture(autouse=True)
def _default_tiles():
    ldni.set_tile_shape(32, 32)
    yield
    ldni.set_tile_shape(0, 0)


@pytest.mark.parametrize("name", sorted(FIXTURES))
def test_exact_fixture_meshes(name):
    v, f, bb, w = FIXTURES[name]
    compare(_run(v, f, bb, w), oracle.sample(v, f, bb, w), bb, label=name)


@pytest.mark.parametrize("w", [1, 2, 33, 77, 128, 131])
def test_icosphere_resolutions(w):
    m = mg.c1_icosphere()
    compare(_run(m.verts, m.tris, m.bbox, w), oracle.sample(m.verts, m.tris, m.bbox, w), m.bbox,
            label=f"c1 w={w}")


@pytest.mark.parametrize("tile", [(8, 1), (16, 16), (64, 16), (256, 4), (32, 32), (8, 64), (0, 0), (8, 8)])
def test_tile_shapes(tile):
    ldni.set_tile_shape(*tile)
    rng = np.random.default_rng(1)
    v, f = mg.concat([mg.uv_flower(48, 96, rng)])
    bb = (-1.4, -1.3, -1.5, 1.4, 1.45, 1.3)
    compare(_run(v, f, bb, 203), oracle.sample(v, f, bb, 203), bb, label=f"tile {tile}")


def _nest(n, level=2):
    rng = np.random.default_rng(3)
    parts = [mg.icosphere(level, 0.95 - 0.04 * k, (0.01, -0.02, 0.015), mg.random_rotation(rng))
             for k in range(n)]
    return mg.concat(parts)


@pytest.mark.parametrize("tile", [(32, 32), (256, 4), (16, 8), (16, 16), (8, 8)])
def test_deep_pixels_chunked_and_oversized_rows(tile):
    """40 layers per ray: the samples of a 32x32 or 256x4 tile do not fit in
    LDS at once, so each tile is written in several runs of pixels."""
    ldni.set_tile_shape(*tile)
    v, f = _nest(20)
    bb = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    ref = oracle.sample(v, f, bb, 256)
    assert max(int(np.diff(r.offsets.astype(np.int64)).max()) for r in ref.values()) == 40
    compare(_run(v, f, bb, 256), ref, bb, label=f"nest tile {tile}")


def test_noncubic_box_and_hits_outside_box():
    """Rays are infinite lines: a mesh sticking out of the box along the axis
    still gives every hit (negative depths, depths beyond hi)."""
    rng = np.random.default_rng(2)
    v, f = mg.concat([mg.icosphere(3, 1.3, (0.2, -0.1, 0.3), mg.random_rotation(rng)),
                      mg.torus(40, 20, 0.5, 0.2, (-0.3, 0.2, -0.2), mg.random_rotation(rng))])
    bb = (-0.9, -1.2, -0.4, 0.8, 1.1, 0.5)
    compare(_run(v, f, bb, 97), oracle.sample(v, f, bb, 97), bb, label="outside")


@pytest.mark.parametrize("scale", [1e-20, 1e-12, 1e12, 3e19])
def test_extreme_coordinate_scales(scale):
    """The walk decides coverage from float32 edge functions where their
    rounding bound allows and falls back to the float64 test elsewhere: tiny
    coordinates (products below the float32 normal range) and huge ones
    (products near or past its largest value) take the fallback or the
    bound's edge, and must still match the oracle bit for bit."""
    rng = np.random.default_rng(11)
    v, f = mg.concat([mg.icosphere(2, 0.8, (0.05, -0.03, 0.02), mg.random_rotation(rng)),
                      mg.torus(24, 12, 0.5, 0.15, (0.1, 0.1, -0.1), mg.random_rotation(rng))])
    v = (v.astype(np.float64) * scale).astype(np.float32)
    bb = tuple(float(np.float32(x * scale)) for x in (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0))
    compare(_run(v, f, bb, 61), oracle.sample(v, f, bb, 61), bb, label=f"scale {scale:g}")


def test_random_meshes_many_axes_masks():
    rng = np.random.default_rng(9)
    for k, axes in enumerate(["x", "y", "z", "xy", "yz", "xz", "xyz"]):
        v, f = mg.concat([mg.icosphere(int(rng.integers(1, 4)), rng.uniform(0.3, 0.9),
                                       rng.uniform(-0.2, 0.2, 3), mg.random_rotation(rng))])
        bb = tuple(rng.uniform(-1.1, -0.95, 3)) + tuple(rng.uniform(0.95, 1.1, 3))
        w = int(rng.integers(20, 150))
        got = _run(v, f, bb, w, axes)
        ref = oracle.sample(v, f, bb, w, axes)
        assert set(got) == set(ref)
        compare(got, ref, bb, label=f"random {k} {axes}")


def test_c1_icosphere_full():
    m = mg.c1_icosphere()
    compare(_run(m.verts, m.tris, m.bbox, m.w), oracle.sample(m.verts, m.tris, m.bbox, m.w), m.bbox,
            label="c1")


def test_c2_flower_full():
    m = mg.c2_flower()
    compare(_run(m.verts, m.tris, m.bbox, m.w), oracle.sample(m.verts, m.tris, m.bbox, m.w), m.bbox,
            label="c2")


def test_c3_scene_rows_sampled():
    """The w=2048 scene at full size; the oracle recomputes a band of rows
    through the 32-layer nest centre and a band near the edge on every axis."""
    m = mg.c3_scene64()
    got = _run(m.verts, m.tris, m.bbox, m.w)
    for a in range(3):
        off, dep, nrm, tri = _np(got[a])
        cnt = np.diff(off.astype(np.int64))
        assert (cnt % 2 == 0).all()
        assert int(cnt.max()) == 32
        for j0, j1 in ((1016, 1032), (100, 108)):
            r = oracle.sample(m.verts, m.tris, m.bbox, m.w, axes=[a], window=(0, m.w, j0, j1))[a]
            s0, s1 = int(off[j0 * m.w]), int(off[j1 * m.w])
            rc = np.diff(r.offsets.astype(np.int64))
            assert np.array_equal(cnt[j0 * m.w:j1 * m.w], rc[j0 * m.w:j1 * m.w])
            assert np.array_equal(tri[s0:s1], r.tri)
            assert np.array_equal(dep[s0:s1].view(np.uint32), r.depth.view(np.uint32))
            assert np.array_equal(nrm[s0:s1].view(np.uint32), r.normal.view(np.uint32))


def test_empty_and_missed_meshes():
    e = _run(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), BOX8, 17)
    for a in range(3):
        assert e[a].n == 0 and int(e[a].offsets.abs().sum()) == 0 and e[a].max_layers == 0
    v, f = mg.concat([mg.box_mesh((20, 20, 20), (21, 21, 21))])
    o = _run(v, f, BOX8, 16)
    for a in range(3):
        assert o[a].n == 0


def test_library_owned_result_matches():
    m = mg.c1_icosphere()
    vt = torch.from_numpy(m.verts).to(DEV)
    ft = torch.from_numpy(m.tris).to(DEV)
    res = ldni.ldni_sample(vt, ft, m.bbox, m.w, "xz")
    ref = oracle.sample(m.verts, m.tris, m.bbox, m.w, "xz")
    got = {a: res.to_torch(a) for a in (0, 2)}
    torch.cuda.synchronize()
    compare(got, ref, m.bbox, label="owned")
    assert res.view(1).n_samples == 0
    res.free()


def test_deterministic_repeat():
    m = mg.c2_flower()
    g1 = _run(m.verts, m.tris, m.bbox, m.w)
    g2 = _run(m.verts, m.tris, m.bbox, m.w)
    for a in range(3):
        for x, y in zip(_np(g1[a]), _np(g2[a])):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


def test_device_detected_errors():
    v, f = mg.concat([mg.box_mesh((1, 1, 1), (2, 2, 2))])
    bad = f.copy()
    bad[5, 2] = 8
    with pytest.raises(ldni.LDNIError) as e:
        _run(v, bad, BOX8, 8)
    assert e.value.code == 2
    bad[5, 2] = -1
    with pytest.raises(ldni.LDNIError) as e:
        _run(v, bad, BOX8, 8)
    assert e.value.code == 2
    vn = v.copy()
    vn[3, 1] = np.inf
    with pytest.raises(ldni.LDNIError) as e:
        _run(vn, f, BOX8, 8)
    assert e.value.code == 6
    # the library keeps working after an error
    compare(_run(v, f, BOX8, 8), oracle.sample(v, f, BOX8, 8), BOX8, label="after error")


def test_pixel_deeper_than_lds_stage():
    """A stack of 2,100 thin boxes: the rays through its middle cross 4,200
    faces, more samples than one place run holds in LDS, so those pixels
    are written to their output ranges and sorted there (a bitonic network
    in global memory)."""
    parts = [mg.box_mesh((3.2, 3.2, 0.5 + 0.003 * k), (4.8, 4.8, 0.5 + 0.003 * k + 0.0015))
             for k in range(2100)]
    v, f = mg.concat(parts)
    ref = oracle.sample(v, f, BOX8, 8, axes="z")
    assert int(np.diff(ref[2].offsets.astype(np.int64)).max()) == 4200
    compare(_run(v, f, BOX8, 8, "z"), ref, BOX8, label="stack")
    ldni.set_tile_shape(8, 2)
    compare(_run(v, f, BOX8, 8, "xyz"), oracle.sample(v, f, BOX8, 8), BOX8, label="stack xyz")


def test_tile_list_retry_on_large_triangles():
    """A dozen triangles spanning thousands of 8x8 tiles overflow the first
    tile-list estimate; the call is redone with the exact size."""
    ldni.set_tile_shape(8, 8)
    v, f = mg.concat([mg.box_mesh((-0.9, -0.95, -0.8), (0.93, 0.9, 0.85))])
    bb = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    for _ in range(2):
        compare(_run(v, f, bb, 1024), oracle.sample(v, f, bb, 1024), bb, label="big triangles")


@pytest.mark.parametrize("tile", [(0, 0), (32, 32)])
def test_staging_capacity_does_not_change_results(tile, monkeypatch):
    """The sampling pass stages hits by tile; tiles that find no room are
    walked again by the write pass.  No staging, a buffer that holds only
    some tiles, and the default buffer all give the oracle's result."""
    ldni.set_tile_shape(*tile)
    m = mg.c2_flower()
    w = 160
    ref = oracle.sample(m.verts, m.tris, m.bbox, w)
    for entries in ("0", "60000", None):
        if entries is None:
            monkeypatch.delenv("LDNI_STAGE_ENTRIES", raising=False)
        else:
            monkeypatch.setenv("LDNI_STAGE_ENTRIES", entries)
        compare(_run(m.verts, m.tris, m.bbox, w), ref, m.bbox, label=f"staging {entries} tile {tile}")


@pytest.mark.parametrize("tile", [(0, 0), (32, 32), (256, 4)])
def test_large_triangles_and_wide_tiles(tile):
    """Large triangles (a box spanning the image at w = 600): every tile-list
    entry covers whole tiles (many candidates per entry), 256-pixel-wide
    tiles included, and a flower mesh adds many entries per tile; both match
    the oracle."""
    ldni.set_tile_shape(*tile)
    v, f = mg.concat([mg.box_mesh((-0.93, -0.91, -0.95), (0.94, 0.92, 0.9))])
    bb = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    compare(_run(v, f, bb, 600), oracle.sample(v, f, bb, 600), bb, label=f"box tile {tile}")
    m = mg.c2_flower()
    compare(_run(m.verts, m.tris, m.bbox, 160), oracle.sample(m.verts, m.tris, m.bbox, 160), m.bbox,
            label=f"flower tile {tile}")


def test_buffers_reused_across_calls_and_results_kept_alive():
    """Calls of different sizes on one stream reuse the buffers earlier calls
    released (the library keeps them per stream), through both the
    torch-output call and the library-owned-output call; results that stay
    alive keep theirs; ldni_trim in between changes nothing."""
    m1 = mg.c1_icosphere()
    m2 = mg.c2_flower()
    cases = [(m1, 128), (m2, 160), (m1, 64), (m2, 96), (m1, 128)]
    refs = {(id(m), w): oracle.sample(m.verts, m.tris, m.bbox, w) for m, w in cases}
    kept = []
    for it, (m, w) in enumerate(cases * 2):
        ref = refs[(id(m), w)]
        if it % 2 == 0:
            compare(_run(m.verts, m.tris, m.bbox, w), ref, m.bbox, label=f"call {it} w={w}")
        else:
            vt = torch.from_numpy(m.verts).to(DEV)
            ft = torch.from_numpy(m.tris).to(DEV)
            r = ldni.ldni_sample(vt, ft, m.bbox, w, "xyz")
            got = {a: r.to_torch(a) for a in range(3)}
            torch.cuda.synchronize()
            compare(got, ref, m.bbox, label=f"owned call {it} w={w}")
            if it % 4 == 1:
                kept.append((r, ref, m.bbox))  # stays alive across later calls
            else:
                r.free()
        if it == 4:
            torch.cuda.synchronize()
            ldni.ldni_trim()
    for r, ref, bb in kept:
        got = {a: r.to_torch(a) for a in range(3)}
        torch.cuda.synchronize()
        compare(got, ref, bb, label="kept result")
        r.free()


@pytest.mark.parametrize("tile", [(16, 16), (32, 32), (8, 8)])
def test_staging_cap_follows_the_deepest_pixel(tile):
    """A stack of 150 thin boxes (300 faces on the rays through it): more hits
    per pixel than the first call's staging cap, so its tiles are walked
    again; later calls of the same shape raise the cap to the deepest pixel
    seen and stage them, and a tile's samples, far more than one place run
    holds, are split into runs taken by several workgroups.  Every call
    gives the oracle's result."""
    ldni.set_tile_shape(*tile)
    parts = [mg.box_mesh((1.1, 1.3, 0.5 + 0.04 * k), (6.7, 6.1, 0.5 + 0.04 * k + 0.02))
             for k in range(150)]
    v, f = mg.concat(parts)
    w = 48
    ref = oracle.sample(v, f, BOX8, w)
    assert int(np.diff(ref[2].offsets.astype(np.int64)).max()) == 300
    for call in range(3):
        compare(_run(v, f, BOX8, w), ref, BOX8, label=f"call {call}")


def test_maximum_resolution_rows_sampled():
    """w = 16384, the largest resolution: the icosphere along z, with the
    oracle recomputing a band of rows through the centre and one near the
    edge of the sphere."""
    m = mg.c1_icosphere()
    w = 16384
    vt = torch.from_numpy(m.verts).to(DEV)
    ft = torch.from_numpy(m.tris).to(DEV)
    got = ldni.sample(vt, ft, m.bbox, w, "z")[2]
    torch.cuda.synchronize()
    for j0, j1 in ((8190, 8194), (1500, 1502)):
        off = got.offsets[j0 * w:j1 * w + 1].cpu().numpy().view(np.uint32).astype(np.int64)
        s0, s1 = int(off[0]), int(off[-1])
        r = oracle.sample(m.verts, m.tris, m.bbox, w, axes="z", window=(0, w, j0, j1))[2]
        rc = np.diff(r.offsets.astype(np.int64))[j0 * w:j1 * w]
        assert np.array_equal(np.diff(off), rc)
        assert np.array_equal(got.tri[s0:s1].cpu().numpy(), r.tri)
        assert np.array_equal(got.depth[s0:s1].cpu().numpy().view(np.uint32), r.depth.view(np.uint32))
        assert np.array_equal(got.normal[s0:s1].cpu().numpy().view(np.uint32), r.normal.view(np.uint32))
    assert got.max_layers == 2


def test_samples_beyond_32_bits_rejected():
    """A stack of 2,100 boxes covering the whole image: 4,200 samples on each
    of the 1,048,576 rays along z, 4.4 x 10^9 in all, more than the u32
    offsets hold.  The call fails with LDNI_ERR_OVERFLOW and the library
    keeps working."""
    parts = [mg.box_mesh((0.01, 0.01, 0.5 + 0.003 * k), (7.99, 7.99, 0.5 + 0.003 * k + 0.0015))
             for k in range(2100)]
    v, f = mg.concat(parts)
    with pytest.raises(ldni.LDNIError) as e:
        _run(v, f, BOX8, 1024, "z")
    assert e.value.code == 4
    m = mg.c1_icosphere()
    compare(_run(m.verts, m.tris, m.bbox, m.w), oracle.sample(m.verts, m.tris, m.bbox, m.w), m.bbox,
            label="after overflow")


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_binning_tables_overflow(tile):
    """Few large triangles at a high resolution: the first chunk of 512
    triangles meets more (image, tile) pairs than its LDS table holds (1,024
    slots), so the binning counts and scatters some tiles through the global
    fallback and the others through the table; the result matches the
    oracle bit for bit."""
    ldni.set_tile_shape(*tile)
    v, f = mg.icosphere(2, radius=0.8, center=(0.03, -0.02, 0.01))
    bb = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    w = 1024
    assert len(f) <= 512
    # distinct (image, tile) pairs of the chunk, from the triangles' bounding boxes
    b = np.asarray(oracle.bbox_f32(bb), np.float64)
    keys = set()
    P = v[f].astype(np.float64)
    for a in range(3):
        u, vv = (a + 1) % 3, (a + 2) % 3
        h = (b[3 + u] - b[u]) / w
        for tri in P:
            i0 = int(np.floor((tri[:, u].min() - b[u]) / h)) // tile[0]
            i1 = int(np.floor((tri[:, u].max() - b[u]) / h)) // tile[0]
            j0 = int(np.floor((tri[:, vv].min() - b[vv]) / h)) // tile[1]
            j1 = int(np.floor((tri[:, vv].max() - b[vv]) / h)) // tile[1]
            keys.update((a, i, j) for i in range(i0, i1 + 1) for j in range(j0, j1 + 1))
    assert len(keys) > 2048
    compare(_run(v, f, bb, w), oracle.sample(v, f, bb, w), bb, label=f"icosphere tile {tile}")
