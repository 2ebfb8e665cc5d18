"""Whole-image parity at the benchmarked sizes, in the launch configuration
that ``bench.py`` times.

* C2 (flower, w = 512) and C3 (scene64, w = 2048): every pixel of all three
  axes from the library-owned one-call ``ldni_sample`` with the automatic
  tile shape, against the oracle (Definitions 1-3: counts, order, triangle
  ids, depth and normal bits).
* C4 (256 meshes, each at its own w): every image of the captured batch is
  byte-identical to its plain ``ldni_sample`` call (compared on the device);
  six meshes (the largest w, the most triangles, four seeded picks) also in
  full against the oracle.
"""
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


def _host(l):
    return (l.offsets.cpu().numpy().view(np.uint32), l.depth.cpu().numpy(), l.normal.cpu().numpy(),
            l.tri.cpu().numpy())


def _against_oracle(got, r, label):
    off, dep, nrm, tri = got
    assert np.array_equal(off, r.offsets), f"{label}: offsets"
    assert np.array_equal(tri, r.tri), f"{label}: triangle ids / order"
    assert np.array_equal(dep.view(np.uint32), r.depth.view(np.uint32)), f"{label}: depth bits"
    assert np.array_equal(nrm.view(np.uint32), r.normal.view(np.uint32)), f"{label}: normal bits"


@pytest.mark.parametrize("which", ["c2_flower", "c3_scene64"])
def test_headline_configs_every_pixel(which):
    m = getattr(mg, which)()
    ldni.set_tile_shape(0, 0)
    v, f = _dev(m.verts, m.tris)
    res = ldni.ldni_sample(v, f, m.bbox, m.w, "xyz")
    for a in range(3):
        got = _host(res.to_torch(a))
        torch.cuda.synchronize()
        ref = oracle.sample(m.verts, m.tris, m.bbox, m.w, axes=[a])[a]
        _against_oracle(got, ref, f"{which} axis {a}")
        cnt = ref.counts
        assert res.view(a).max_layers == int(cnt.max())
        assert res.view(a).n_samples == ref.n
        del got, ref
    res.free()


def _bytes_equal(x: torch.Tensor, y: torch.Tensor) -> bool:
    if x.shape != y.shape:
        return False
    return bool(torch.equal(x.contiguous().view(torch.uint8), y.contiguous().view(torch.uint8)))


def test_batch256_every_image_equals_plain_calls():
    meshes = mg.c4_batch256()
    dev = [_dev(m.verts, m.tris) for m in meshes]
    b = ldni.sample_batch([(v, f, m.bbox, m.w) for (v, f), m in zip(dev, meshes)], "xyz")
    ldni.set_tile_shape(0, 0)
    for k, ((v, f), m) in enumerate(zip(dev, meshes)):
        plain = ldni.ldni_sample(v, f, m.bbox, m.w, "xyz")
        for a in range(3):
            x, y = b.to_torch(k, a), plain.to_torch(a)
            label = f"mesh {k} (w {m.w}, {m.n_tris} triangles) axis {a}"
            for name in ("offsets", "depth", "normal", "tri"):
                assert _bytes_equal(getattr(x, name), getattr(y, name)), f"{label}: {name}"
            assert b.view(k, a).max_layers == plain.view(a).max_layers, label
        plain.free()
    rng = np.random.default_rng(3)
    picks = {int(np.argmax([m.w for m in meshes])), int(np.argmax([m.n_tris for m in meshes]))}
    picks |= {int(k) for k in rng.choice(len(meshes), 4, replace=False)}
    for k in sorted(picks):
        m = meshes[k]
        for a in range(3):
            got = _host(b.to_torch(k, a))
            ref = oracle.sample(m.verts, m.tris, m.bbox, m.w, axes=[a])[a]
            _against_oracle(got, ref, f"mesh {k} (w {m.w}, {m.n_tris} triangles) axis {a}")
    b.free()
