"""Central finite differences of the squared-error LDNI loss used for the
differentiation checks, evaluated with the oracle's float64 sampling.

The loss is L = sum over axes, over pixels whose sample count equals the
target's, of sum_k (d_k - d*_k)^2 + |n_k - n*_k|^2 (sample k paired with
target sample k).  Moving one vertex only changes samples inside the pixel
window of its adjacent triangles, so each difference is taken over that
window; a vertex whose (pixel, triangle) sequence changes at +-h, or whose
float64 sequence differs from the float32 one the pairing came from, is
skipped.
"""
from __future__ import annotations

import numpy as np

import oracle


def pairing(ref_off, tgt_off):
    """(sample index, target sample index, pixel mask) of the count-matched
    pixels, k-th sample paired with k-th."""
    ref_off = np.asarray(ref_off).astype(np.int64)
    tgt_off = np.asarray(tgt_off).astype(np.int64)
    c = np.diff(ref_off)
    ct = np.diff(tgt_off)
    mask = (c == ct) & (c > 0)
    pix = np.nonzero(mask)[0]
    cnt = c[pix]
    k = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    s = np.repeat(ref_off[pix], cnt) + k
    st = np.repeat(tgt_off[pix], cnt) + k
    return s, st, mask


def _window_loss(v64, tris, bbox, w, a, win, mask, tgt_depth, tgt_normal, tgt_off, sel=None):
    """sel: ids of the triangles that can reach the window (all if None);
    triangle ids in the returned keys are the mesh's own."""
    sub = tris if sel is None else tris[sel]
    r = oracle.sample_f64(v64, sub, bbox, w, a, window=win)
    if sel is not None:
        r.tri = sel[r.tri].astype(np.int32)
    off = r.offsets.astype(np.int64)
    i0, i1, j0, j1 = win
    L = 0.0
    keys = []
    for j in range(j0, j1):
        for i in range(i0, i1):
            p = j * w + i
            s0, s1 = off[p], off[p + 1]
            keys += [(p, int(t)) for t in r.tri[s0:s1]]
            if not mask[p]:
                continue
            t0 = int(tgt_off[p])
            d = r.depth[s0:s1] - tgt_depth[t0:t0 + s1 - s0]
            n = r.normal[s0:s1] - tgt_normal[t0:t0 + s1 - s0]
            L += float((d * d).sum() + (n * n).sum())
    return L, keys


def finite_differences(verts, tris, bbox, w, tgt, n_vertices=64, seed=4, h=1e-6, max_tries=400):
    """FD gradients of the loss at n_vertices random vertices.

    tgt: {axis: (offsets u32 [w*w+1], depth f32 [n], normal f32 [n,3])} of the
    target LDNI.  Returns (vertex ids, fd [k,3])."""
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.int32)
    v64 = verts.astype(np.float64)
    f32 = oracle.sample(verts, tris, bbox, w)
    masks = {a: pairing(f32[a].offsets, tgt[a][0])[2] for a in range(3)}
    adj = [[] for _ in range(len(verts))]
    for t, tri in enumerate(tris):
        for q in tri:
            adj[int(q)].append(t)
    bb = np.asarray(oracle.bbox_f32(bbox))
    lo, hpix = bb[:3], (bb[3:] - bb[:3]) / w
    Pt = v64[tris]                                    # [T,3,3]
    tmin, tmax = Pt.min(1), Pt.max(1)                 # [T,3]

    def reach(a, win):
        # triangles whose projection can cover a pixel centre of the window
        # (one pixel of margin beyond any perturbation of +-h)
        u, vv = (a + 1) % 3, (a + 2) % 3
        i0, i1, j0, j1 = win
        ulo, uhi = lo[u] + (i0 - 1) * hpix[u], lo[u] + (i1 + 1) * hpix[u]
        vlo, vhi = lo[vv] + (j0 - 1) * hpix[vv], lo[vv] + (j1 + 1) * hpix[vv]
        return np.nonzero((tmax[:, u] >= ulo) & (tmin[:, u] <= uhi) &
                          (tmax[:, vv] >= vlo) & (tmin[:, vv] <= vhi))[0]
    rng = np.random.default_rng(seed)
    ids, fds = [], []
    tries = 0
    while len(ids) < n_vertices and tries < max_tries:
        tries += 1
        vid = int(rng.integers(0, len(verts)))
        P = v64[tris[adj[vid]].ravel()]
        fd = np.zeros(3)
        ok = True
        wins = []
        for a in range(3):
            u, vv = (a + 1) % 3, (a + 2) % 3
            wins.append((max(0, int(np.floor((P[:, u].min() - lo[u]) / hpix[u])) - 2),
                         min(w, int(np.ceil((P[:, u].max() - lo[u]) / hpix[u])) + 2),
                         max(0, int(np.floor((P[:, vv].min() - lo[vv]) / hpix[vv])) - 2),
                         min(w, int(np.ceil((P[:, vv].max() - lo[vv]) / hpix[vv])) + 2)))
        sels = [reach(a, wins[a]) for a in range(3)]
        # the float64 sample sequence must be the float32 one the pairing used
        for a in range(3):
            i0, i1, j0, j1 = wins[a]
            off = f32[a].offsets.astype(np.int64)
            k32 = [(j * w + i, int(t)) for j in range(j0, j1) for i in range(i0, i1)
                   for t in f32[a].tri[off[j * w + i]:off[j * w + i + 1]]]
            _, k64 = _window_loss(v64, tris, bbox, w, a, wins[a], masks[a], tgt[a][1], tgt[a][2],
                                  tgt[a][0].astype(np.int64), sels[a])
            if k64 != k32:
                ok = False
                break
        if not ok:
            continue
        for c in range(3):
            Lp = Lm = 0.0
            for a in range(3):
                T = (masks[a], tgt[a][1].astype(np.float64), tgt[a][2].astype(np.float64),
                     tgt[a][0].astype(np.int64))
                _, k0 = _window_loss(v64, tris, bbox, w, a, wins[a], *T, sels[a])
                vp, vm = v64.copy(), v64.copy()
                vp[vid, c] += h
                vm[vid, c] -= h
                lp, kp = _window_loss(vp, tris, bbox, w, a, wins[a], *T, sels[a])
                lm, km = _window_loss(vm, tris, bbox, w, a, wins[a], *T, sels[a])
                if kp != k0 or km != k0:
                    ok = False
                    break
                Lp += lp
                Lm += lm
            if not ok:
                break
            fd[c] = (Lp - Lm) / (2 * h)
        if ok:
            ids.append(vid)
            fds.append(fd)
    return np.array(ids, dtype=np.int64), np.array(fds)


def upstream_grads(ref, tgt):
    """dL/d depth and dL/d normal per axis for the loss: 2(d - d*) and
    2(n - n*) on paired samples, zero elsewhere.  ref/tgt: {axis: (offsets,
    depth, normal)} as numpy arrays."""
    gd, gn = {}, {}
    for a in ref:
        s, st, _ = pairing(ref[a][0], tgt[a][0])
        g1 = np.zeros(len(ref[a][1]), np.float32)
        g3 = np.zeros((len(ref[a][1]), 3), np.float32)
        g1[s] = 2.0 * (ref[a][1][s].astype(np.float64) - tgt[a][1][st])
        g3[s] = 2.0 * (ref[a][2][s].astype(np.float64) - tgt[a][2][st])
        gd[a], gn[a] = g1, g3
    return gd, gn
