"""ldni_backward_noalloc (for callers that cannot allocate device memory)
against ldni_backward: the same vertex gradients, through the C ABI, on two
calls in a row (the flower mesh, then a smaller icosphere on fewer axes), a
third with every library allocation failing, and the size limit."""
import numpy as np
import pytest
import torch

import paper_1009_0794_amd as ldni
from paper_1009_0794_amd import meshgen as mg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _grads(res, seed):
    """Seeded upstream gradients for every sample of a forward result."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    gd, gn = {}, {}
    for a, l in res.items():
        n = int(l.tri.shape[0])
        gd[a] = torch.randn(n, generator=g).to(DEV)
        gn[a] = torch.randn(n, 3, generator=g).to(DEV)
    return gd, gn


def _both(m, w, axes, seed):
    v = torch.from_numpy(m.verts).to(DEV)
    f = torch.from_numpy(m.tris).to(DEV)
    res = ldni.sample(v, f, m.bbox, w, axes)
    gd, gn = _grads(res, seed)
    ref = ldni.ldni_backward(v, f, m.bbox, w, res, gd, gn)
    got = ldni.ldni_backward(v, f, m.bbox, w, res, gd, gn, no_alloc=True)
    torch.cuda.synchronize()
    return ref.cpu().numpy().astype(np.float64), got.cpu().numpy().astype(np.float64)


def _close(ref, got, label):
    # The two calls run the same kernels on the same data; only the order of
    # the float32 atomic additions differs.  A vertex sums a few hundred
    # terms, so their float32 rounding differences stay far below 1e-5 of
    # the largest gradient.
    scale = float(np.abs(ref).max())
    assert scale > 0.0, label
    assert np.abs(got - ref).max() <= 1e-5 * scale, label


def test_noalloc_backward_matches_backward(monkeypatch):
    flower = mg.c2_flower()
    assert flower.n_tris <= 262144
    ref, got = _both(flower, 512, "xyz", 1)
    _close(ref, got, "flower, first call")
    # a second call with a smaller input: the scratch still holds the
    # flower's sums and must be cleared
    ico = mg.c1_icosphere()
    ref, got = _both(ico, 128, "xz", 2)
    _close(ref, got, "icosphere, second call")
    # with every library allocation failing, the no-allocation call still works
    v = torch.from_numpy(ico.verts).to(DEV)
    f = torch.from_numpy(ico.tris).to(DEV)
    res = ldni.sample(v, f, ico.bbox, 96, "y")
    gd, gn = _grads(res, 3)
    ref3 = ldni.ldni_backward(v, f, ico.bbox, 96, res, gd, gn).cpu().numpy().astype(np.float64)
    monkeypatch.setenv("LDNI_FAULT", "alloc")
    got3 = ldni.ldni_backward(v, f, ico.bbox, 96, res, gd, gn, no_alloc=True)
    torch.cuda.synchronize()
    monkeypatch.delenv("LDNI_FAULT")
    _close(ref3, got3.cpu().numpy().astype(np.float64), "icosphere, allocations failing")


def test_noalloc_backward_rejects_too_many_triangles():
    parts = [mg.icosphere(5, 0.1 + 0.001 * k, (0.0, 0.0, 0.0), np.eye(3)) for k in range(13)]
    v, f = mg.concat(parts)
    assert len(f) > 262144
    vt = torch.from_numpy(v).to(DEV)
    ft = torch.from_numpy(f).to(DEV)
    bb = (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)
    res = ldni.sample(vt, ft, bb, 32, "z")
    with pytest.raises(ldni.LDNIError) as e:
        ldni.ldni_backward(vt, ft, bb, 32, res, {2: torch.ones(res[2].n, device=DEV)}, None, no_alloc=True)
    assert e.value.code == 1
