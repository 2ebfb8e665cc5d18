"""The differentiable sampler's vertex gradients on the GPU.

Checked against the oracle's float64 analytic gradient (itself pinned by
finite differences on the CPU), against translation identities, and on the
flower workload against float64 central finite differences of the sampling
definition (the oracle's float64 variant) for a squared-error loss to the
LDNI of a perturbed copy.
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


def _generic(seed):
    rng = np.random.default_rng(seed)
    v, f = mg.concat([mg.icosphere(3, 0.8, (0.05, -0.03, 0.02), mg.random_rotation(rng)),
                      mg.torus(48, 24, 0.45, 0.15, (0.1, 0.2, -0.1), mg.random_rotation(rng))])
    return v, f, (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0)


@pytest.mark.parametrize("w", [24, 97])
def test_backward_matches_oracle_gradient(w):
    v, f, bb = _generic(w)
    vt, ft = _dev(v, f)
    res = ldni.sample(vt, ft, bb, w, "xyz")
    rng = np.random.default_rng(100 + w)
    gd = {a: rng.normal(size=res[a].n).astype(np.float32) for a in res}
    gn = {a: rng.normal(size=(res[a].n, 3)).astype(np.float32) for a in res}
    g = ldni.ldni_backward(vt, ft, bb, w, res,
                           {a: torch.from_numpy(x).to(DEV) for a, x in gd.items()},
                           {a: torch.from_numpy(x).to(DEV) for a, x in gn.items()})
    g = g.cpu().numpy().astype(np.float64)
    ref = np.zeros_like(g)
    orc = oracle.sample(v, f, bb, w)
    for a in range(3):
        ref += oracle.backward(v, f, bb, w, a, orc[a], gd[a], gn[a])
    scale = np.abs(ref).max()
    assert np.abs(g - ref).max() <= 1e-4 * scale, np.abs(g - ref).max() / scale


@pytest.mark.parametrize("name", ["box_on_centres", "polycube_on_centres", "lattice_hull"])
def test_backward_vertices_on_centres_across_tile_borders(name):
    """Meshes whose vertices sit on pixel centres, moved so that they span the
    border between 16-pixel tiles (centres 15.5 and 16.5 of a 32-pixel grid):
    a tile stores a triangle's sums with plain stores only when every pixel
    that can hold its samples is in the tile, so triangles ending exactly on
    the centres next to the border must still get every contribution."""
    from tests.golden.fixture_meshes import FIXTURES
    v0, f, _, _ = FIXTURES[name]
    v = (np.asarray(v0, np.float64) + 12.0).astype(np.float32)
    bb, w = (0.0, 0.0, 0.0, 32.0, 32.0, 32.0), 32
    vt, ft = _dev(v, f)
    res = ldni.sample(vt, ft, bb, w, "xyz")
    rng = np.random.default_rng(7)
    gd = {a: rng.normal(size=res[a].n).astype(np.float32) for a in res}
    gn = {a: rng.normal(size=(res[a].n, 3)).astype(np.float32) for a in res}
    g = ldni.ldni_backward(vt, ft, bb, w, res,
                           {a: torch.from_numpy(x).to(DEV) for a, x in gd.items()},
                           {a: torch.from_numpy(x).to(DEV) for a, x in gn.items()})
    g = g.cpu().numpy().astype(np.float64)
    ref = np.zeros_like(g)
    orc = oracle.sample(v, f, bb, w)
    for a in range(3):
        assert res[a].n == orc[a].n
        ref += oracle.backward(v, f, bb, w, a, orc[a], gd[a], gn[a])
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(g - ref).max() <= 1e-4 * scale, np.abs(g - ref).max() / scale


def test_backward_accumulates_and_axes_optional():
    v, f, bb = _generic(5)
    vt, ft = _dev(v, f)
    res = ldni.sample(vt, ft, bb, 40, "xz")
    gd = {0: torch.ones(res[0].n, device=DEV)}
    g1 = ldni.ldni_backward(vt, ft, bb, 40, res, gd, None)
    g2 = ldni.ldni_backward(vt, ft, bb, 40, res, gd, None, grad_verts=g1.clone())
    torch.cuda.synchronize()
    assert torch.allclose(g2, 2 * g1, rtol=1e-5, atol=1e-6)
    # depth along x moves with a translation along x: sum of x gradients = sum gd
    assert abs(float(g1[:, 0].double().sum()) - res[0].n) <= 1e-3 * res[0].n
    # no gradient at all leaves grad_verts untouched
    z = ldni.ldni_backward(vt, ft, bb, 40, res, None, None)
    assert float(z.abs().sum()) == 0.0


def test_translation_identities_gpu():
    v, f, bb = _generic(6)
    vt, ft = _dev(v, f)
    res = ldni.sample(vt, ft, bb, 64, "xyz")
    rng = np.random.default_rng(1)
    for a in range(3):
        gd = torch.from_numpy(rng.normal(size=res[a].n).astype(np.float32)).to(DEV)
        g = ldni.ldni_backward(vt, ft, bb, 64, {a: res[a]}, {a: gd}, None).double().sum(0)
        n = res[a].normal.double()
        expect = (gd.double()[:, None] * n / n[:, a:a + 1]).sum(0)
        assert torch.allclose(g, expect, rtol=1e-4, atol=1e-4 * float(expect.abs().max()))
        gn = torch.from_numpy(rng.normal(size=(res[a].n, 3)).astype(np.float32)).to(DEV)
        gnorm = ldni.ldni_backward(vt, ft, bb, 64, {a: res[a]}, None, {a: gn})
        assert float(gnorm.double().sum(0).abs().max()) <= 1e-4 * float(gnorm.abs().max())


def test_autograd_function_matches_direct_call():
    v, f, bb = _generic(7)
    vt, ft = _dev(v, f)
    vt.requires_grad_(True)
    out = ldni.sample_diff(vt, ft, bb, 50, "xyz")
    loss = sum((out[a].depth ** 2).sum() + (out[a].normal[:, 0] * 0.5).sum() for a in out)
    loss.backward()
    with torch.no_grad():
        res = ldni.sample(vt.detach(), ft, bb, 50, "xyz")
        g = ldni.ldni_backward(vt.detach(), ft, bb, 50, res, {a: 2 * res[a].depth for a in res},
                               {a: torch.tensor([0.5, 0.0, 0.0], device=DEV).expand(res[a].n, 3)
                                for a in res})
    assert torch.allclose(vt.grad, g, rtol=1e-4, atol=1e-5 * float(g.abs().max()))
    for a in out:
        assert not out[a].offsets.requires_grad and not out[a].tri.requires_grad


# --------------------------------------------------------------- flower + FD

def test_flower_loss_gradient_against_finite_differences():
    """Flower 512x256 at w=512; loss = sum (d - d*)^2 + |n - n*|^2 over pixels
    whose count equals the target's (the LDNI of a radially perturbed copy,
    N(0, 0.005), seed 3); the gradient from the autograd function at 64
    random vertices (seed 4) against float64 central differences, h = 1e-6."""
    from tests import fdcheck
    m = mg.c2_flower()
    tgt_mesh = mg.c5_target(m)
    w, bb = m.w, m.bbox
    vt, ft = _dev(m.verts, m.tris)
    tv, _ = _dev(tgt_mesh.verts, tgt_mesh.tris)
    tgt_gpu = ldni.sample(tv, ft, bb, w, "xyz")
    vt.requires_grad_(True)
    out = ldni.sample_diff(vt, ft, bb, w, "xyz")
    loss = 0.0
    T = {}
    for a in range(3):
        ref_off = out[a].offsets.detach().cpu().numpy().view(np.uint32)
        tgt_off = tgt_gpu[a].offsets.cpu().numpy().view(np.uint32)
        s, st, _ = fdcheck.pairing(ref_off, tgt_off)
        si, sti = torch.from_numpy(s).to(DEV), torch.from_numpy(st).to(DEV)
        dd = out[a].depth[si] - tgt_gpu[a].depth[sti]
        dn = out[a].normal[si] - tgt_gpu[a].normal[sti]
        loss = loss + (dd * dd).sum() + (dn * dn).sum()
        T[a] = (tgt_off, tgt_gpu[a].depth.cpu().numpy(), tgt_gpu[a].normal.cpu().numpy())
    loss.backward()
    g = vt.grad.cpu().numpy().astype(np.float64)
    ids, fd = fdcheck.finite_differences(m.verts, m.tris, bb, w, T, n_vertices=64, seed=4)
    assert len(ids) == 64, f"only {len(ids)} usable vertices"
    got = g[ids]
    tol = 1e-3 * np.abs(fd) + 1e-4 * np.abs(fd).max()
    assert (np.abs(got - fd) <= tol).all(), np.max(np.abs(got - fd) / tol)
