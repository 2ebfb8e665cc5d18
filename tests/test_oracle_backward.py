"""Pins of the oracle's analytic vertex gradient.

The loss is linear in the samples, L = sum gd_s * depth_s + gn_s . n_s, so its
gradient is what the differentiable sampler must produce for upstream grads
(gd, gn).  It is checked against float64 central finite differences of the
sampling definition itself (the float64 oracle), on sample sets that do not
change at +-h, and against translation identities.
"""
import numpy as np
import pytest

import oracle
from paper_1009_0794_amd import meshgen as mg


def _mesh(seed=0):
    rng = np.random.default_rng(seed)
    v, f = mg.concat([mg.icosphere(2, 0.8, (0.05, -0.03, 0.02), mg.random_rotation(rng))])
    return v, f, (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0), 24


def _keyed(ax):
    pix = np.repeat(np.arange(ax.w * ax.w), np.diff(ax.offsets.astype(np.int64)))
    return {(int(p), int(t)): k for k, (p, t) in enumerate(zip(pix, ax.tri))}


def _loss64(v64, f, bb, w, axis, keys, gd, gn):
    ax = oracle.sample_f64(v64, f, bb, w, axis)
    k2 = _keyed(ax)
    assert set(k2) == set(keys), "sample set changed under the perturbation"
    L = 0.0
    for key, s in keys.items():
        s2 = k2[key]
        L += float(gd[s]) * ax.depth[s2] + float(np.dot(gn[s], ax.normal[s2]))
    return L


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_backward_matches_central_differences(axis):
    v, f, bb, w = _mesh(axis)
    ref = oracle.sample(v, f, bb, w, axes=[axis])[axis]
    keys = _keyed(ref)
    rng = np.random.default_rng(10 + axis)
    gd = rng.normal(size=ref.n).astype(np.float32)
    gn = rng.normal(size=(ref.n, 3)).astype(np.float32)
    g = oracle.backward(v, f, bb, w, axis, ref, gd, gn)
    v64 = v.astype(np.float64)
    h = 1e-6
    checked = 0
    for vid in rng.choice(len(v), size=12, replace=False):
        for c in range(3):
            vp, vm = v64.copy(), v64.copy()
            vp[vid, c] += h
            vm[vid, c] -= h
            try:
                fd = (_loss64(vp, f, bb, w, axis, keys, gd, gn)
                      - _loss64(vm, f, bb, w, axis, keys, gd, gn)) / (2 * h)
            except AssertionError:
                continue
            assert abs(g[vid, c] - fd) <= 1e-5 * abs(fd) + 1e-6 * max(1.0, np.abs(g).max()), (vid, c)
            checked += 1
    assert checked >= 30


def test_translation_identities():
    """Moving every vertex by t shifts each depth by t_a and leaves normals
    unchanged: sum_v dL/dv = sum_s gd_s n_s / n_{s,a} for the depth term and 0
    for the normal term."""
    v, f, bb, w = _mesh(3)
    for axis in range(3):
        ref = oracle.sample(v, f, bb, w, axes=[axis])[axis]
        rng = np.random.default_rng(axis)
        gd = rng.normal(size=ref.n).astype(np.float32)
        gn = rng.normal(size=(ref.n, 3)).astype(np.float32)
        gdep = oracle.backward(v, f, bb, w, axis, ref, gd, None)
        n = ref.normal.astype(np.float64)
        expect = (gd[:, None].astype(np.float64) * n / n[:, axis:axis + 1]).sum(0)
        np.testing.assert_allclose(gdep.sum(0), expect, rtol=1e-5, atol=1e-9)
        # depth along the axis moves rigidly with a translation along it
        assert gdep.sum(0)[axis] == pytest.approx(float(gd.astype(np.float64).sum()), rel=1e-9, abs=1e-9)
        gnrm = oracle.backward(v, f, bb, w, axis, ref, None, gn)
        assert np.abs(gnrm.sum(0)).max() <= 1e-9 * max(1.0, np.abs(gnrm).max())


def test_normal_gradient_is_tangent():
    """n is scale-invariant in N, so scaling the mesh about the origin changes
    no normal: sum_v v . dL/dv = 0 for a normal-only loss."""
    v, f, bb, w = _mesh(4)
    ref = oracle.sample(v, f, bb, w, axes=[2])[2]
    gn = np.random.default_rng(1).normal(size=(ref.n, 3)).astype(np.float32)
    g = oracle.backward(v, f, bb, w, 2, ref, None, gn)
    assert abs(float((g * v.astype(np.float64)).sum())) <= 1e-9 * max(1.0, np.abs(g).sum())


def test_loss_gradient_harness_on_small_flower():
    """The finite-difference harness used for the flower workload, checked
    with the oracle's own analytic gradient on a reduced flower."""
    from tests import fdcheck
    rng = np.random.default_rng(0)
    v, f = mg.concat([mg.uv_flower(24, 48, rng)])
    base = mg.Mesh(v, f, (-1.4, -1.4, -1.4, 1.4, 1.4, 1.4), 96)
    tgt_mesh = mg.c5_target(base)
    w, bb = base.w, base.bbox
    ref = oracle.sample(v, f, bb, w)
    tgt = oracle.sample(tgt_mesh.verts, f, bb, w)
    R = {a: (ref[a].offsets, ref[a].depth, ref[a].normal) for a in range(3)}
    T = {a: (tgt[a].offsets, tgt[a].depth, tgt[a].normal) for a in range(3)}
    gd, gn = fdcheck.upstream_grads(R, T)
    g = sum(oracle.backward(v, f, bb, w, a, ref[a], gd[a], gn[a]) for a in range(3))
    ids, fd = fdcheck.finite_differences(v, f, bb, w, T, n_vertices=16, seed=4)
    assert len(ids) == 16
    got = g[ids]
    tol = 1e-3 * np.abs(fd) + 1e-4 * np.abs(fd).max()
    assert (np.abs(got - fd) <= tol).all(), np.max(np.abs(got - fd) / tol)
