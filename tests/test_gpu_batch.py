"""Batched sampling: many meshes with their own resolutions and tile shapes
in one captured graph must give, mesh by mesh, exactly the single-mesh
results (which are themselves checked against the oracle)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1009_0794_amd as ldni
from paper_1009_0794_amd import meshgen as mg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(v, f):
    return (torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(f, np.int32)).to(DEV))


def _np(l):
    return (l.offsets.cpu().numpy().view(np.uint32), l.depth.cpu().numpy(), l.normal.cpu().numpy(),
            l.tri.cpu().numpy())


def _same(a, b, label):
    for x, y, name in zip(_np(a), _np(b), ("offsets", "depth", "normal", "tri")):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"{label}: {name}"
    assert a.max_layers == b.max_layers, label


def _small_batch(n=12, seed=5):
    ms = mg.c4_batch256(seed=seed, n=n, t_lo=200, t_hi=20000)
    rng = np.random.default_rng(seed)
    tiles = [(32, 32), (16, 16), (64, 16), (8, 8), None]
    out = []
    for m in ms:
        w = int(rng.choice([17, 64, 100, 128, 257]))
        out.append((m, w, tiles[int(rng.integers(0, len(tiles)))]))
    return out


def test_batch_equals_single_mesh_calls():
    items = _small_batch()
    dev = [(_dev(m.verts, m.tris), m, w, t) for m, w, t in items]
    b = ldni.sample_batch([(v, f, m.bbox, w, t) for (v, f), m, w, t in dev], "xyz")
    for k, ((v, f), m, w, t) in enumerate(dev):
        ldni.set_tile_shape(*(t or (0, 0)))
        single = ldni.sample(v, f, m.bbox, w, "xyz")
        for a in range(3):
            _same(b.to_torch(k, a), single[a], f"mesh {k} axis {a}")
    ldni.set_tile_shape(0, 0)
    # one mesh against the oracle directly
    m, w = items[0][0], items[0][1]
    ref = oracle.sample(m.verts, m.tris, m.bbox, w)
    for a in range(3):
        off, dep, nrm, tri = _np(b.to_torch(0, a))
        assert np.array_equal(off, ref[a].offsets) and np.array_equal(tri, ref[a].tri)
        assert np.array_equal(dep.view(np.uint32), ref[a].depth.view(np.uint32))
    b.free()


def test_graph_replays_with_eager_work_between():
    items = _small_batch(6, seed=8)
    dev = [(_dev(m.verts, m.tris), m, w, t) for m, w, t in items]
    b = ldni.sample_batch([(v, f, m.bbox, w, t) for (v, f), m, w, t in dev], "xz")
    first = {(k, a): b.to_torch(k, a) for k in range(len(dev)) for a in (0, 2)}
    torch.cuda.synchronize()
    for r in range(3):
        x = torch.randn(1 << 20, device=DEV)
        (x * 2).sum().item()  # unrelated eager work and a synchronisation
        b.run()
        for k in range(len(dev)):
            for a in (0, 2):
                _same(b.to_torch(k, a), first[(k, a)], f"replay {r} mesh {k} axis {a}")
            assert b.view(k, 1).n_samples == 0
    b.free()


def test_batch_follows_changed_vertices_and_regrows():
    """Runs sample the current vertex contents; a larger mesh extent needs
    more samples and larger tile lists, so the buffers grow and the graph is
    captured again."""
    items = _small_batch(4, seed=9)
    dev = [(_dev(m.verts, m.tris), m, w, t) for m, w, t in items]
    b = ldni.sample_batch([(v, f, m.bbox, w, t) for (v, f), m, w, t in dev], "xyz")
    for (v, f), m, w, t in dev:
        v.mul_(1.6)  # grows each mesh within its padded box (and beyond it)
    b.run()
    for k, ((v, f), m, w, t) in enumerate(dev):
        ldni.set_tile_shape(*(t or (0, 0)))
        single = ldni.sample(v, f, m.bbox, w, "xyz")
        for a in range(3):
            _same(b.to_torch(k, a), single[a], f"scaled mesh {k} axis {a}")
    ldni.set_tile_shape(0, 0)
    b.free()


def test_batch_reports_device_errors():
    v, f = mg.concat([mg.box_mesh((1, 1, 1), (2, 2, 2))])
    bad = f.copy()
    bad[0, 0] = 99
    good = _dev(v, f)
    badd = _dev(v, bad)
    with pytest.raises(ldni.LDNIError) as e:
        ldni.sample_batch([(good[0], good[1], (0, 0, 0, 8, 8, 8), 8),
                           (badd[0], badd[1], (0, 0, 0, 8, 8, 8), 16)])
    assert e.value.code == 2


def test_full_batch256_rows_against_oracle():
    """The timed batch at full size: the 256 seeded meshes (log-uniform
    triangle counts, each at its own w, tile shapes from the tuned table) in
    one graph.  Every pixel count is even (the meshes are closed); for six
    meshes (the largest w, the most triangles and four seeded picks) an
    8-row band through the middle of every axis equals the oracle bit for
    bit; a second replay writes the same bytes."""
    meshes = mg.c4_batch256()
    dev = [_dev(m.verts, m.tris) for m in meshes]
    b = ldni.sample_batch([(v, f, m.bbox, m.w) for (v, f), m in zip(dev, meshes)], "xyz")
    for k in range(len(meshes)):
        for a in range(3):
            off = b.to_torch(k, a).offsets.to(torch.int64) & 0xFFFFFFFF
            assert bool(((off[1:] - off[:-1]) % 2 == 0).all()), f"mesh {k} axis {a}: odd count"
    rng = np.random.default_rng(3)
    picks = {int(np.argmax([m.w for m in meshes])), int(np.argmax([m.n_tris for m in meshes]))}
    picks |= {int(k) for k in rng.choice(len(meshes), 4, replace=False)}
    first = {}
    for k in sorted(picks):
        m = meshes[k]
        j0, j1 = max(m.w // 2 - 4, 0), min(m.w // 2 + 4, m.w)
        for a in range(3):
            off, dep, nrm, tri = _np(b.to_torch(k, a))
            first[(k, a)] = [x.copy() for x in (off, dep, nrm, tri)]
            cnt = np.diff(off.astype(np.int64))
            r = oracle.sample(m.verts, m.tris, m.bbox, m.w, axes=[a], window=(0, m.w, j0, j1))[a]
            rc = np.diff(r.offsets.astype(np.int64))
            s0, s1 = int(off[j0 * m.w]), int(off[j1 * m.w])
            label = f"mesh {k} (w {m.w}, {m.n_tris} triangles) axis {a}"
            assert np.array_equal(cnt[j0 * m.w:j1 * m.w], rc[j0 * m.w:j1 * m.w]), label
            assert np.array_equal(tri[s0:s1], r.tri), label
            assert np.array_equal(dep[s0:s1].view(np.uint32), r.depth.view(np.uint32)), label
            assert np.array_equal(nrm[s0:s1].view(np.uint32), r.normal.view(np.uint32)), label
    b.run()
    torch.cuda.synchronize()
    for (k, a), want in first.items():
        for x, y in zip(_np(b.to_torch(k, a)), want):
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), f"replay: mesh {k} axis {a}"
    b.free()
