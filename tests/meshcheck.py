"""Mesh checks used by the tests: closedness, orientation and the
divergence-theorem volume (the quantity the LDNI's inside intervals measure,
Sec. 2 after Proposition 1)."""
from __future__ import annotations

import numpy as np


def is_closed_oriented(tris) -> bool:
    """Every directed edge occurs exactly once and its reverse exactly once."""
    t = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    key = e[:, 0] * (int(e.max()) + 1) + e[:, 1]
    rkey = e[:, 1] * (int(e.max()) + 1) + e[:, 0]
    uniq, cnt = np.unique(key, return_counts=True)
    if (cnt != 1).any():
        return False
    return bool(np.isin(rkey, uniq).all())


def volume(verts, tris) -> float:
    """(1/6) sum A . (B x C) in float64."""
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int64)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def ldni_volume(ax, bbox, axis) -> float:
    """Sum over pixels of the inside intervals (odd-th to next even-th depth)
    times the pixel area."""
    u, v = (axis + 1) % 3, (axis + 2) % 3
    w = ax.w
    bb = np.asarray(bbox, np.float32).astype(np.float64)
    area = (bb[3 + u] - bb[u]) / w * (bb[3 + v] - bb[v]) / w
    d = ax.depth.astype(np.float64)
    off = ax.offsets.astype(np.int64)
    cnt = np.diff(off)
    assert (cnt % 2 == 0).all()
    # samples alternate enter/leave: sum(d[odd]) - sum(d[even]) per pixel
    sign = np.ones(len(d))
    idx = np.arange(len(d)) - np.repeat(off[:-1], cnt)
    sign[idx % 2 == 0] = -1.0
    return float((sign * d).sum() * area)
