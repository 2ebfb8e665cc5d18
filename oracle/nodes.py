"""TEST INFRASTRUCTURE ONLY: CPU oracle for the inside/outside classification
of grid nodes from three LDNIs.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product library shares no code with it.

Method (Definition 3; Sec. 5.1, step 1 of the contouring algorithm): the
rays of the x-, y- and z-LDNI of one box at one resolution w meet at the
nodes of a w x w x w grid.  Along each of its three rays a node is inside
the solid when it lies in one of the ray's volumes, the stretch from a
sample of odd rank to the next sample (ranks counted from 1; Sec. 2 after
Proposition 1).  Numerical error and degenerate configurations can make the
three rays disagree, so a node is classified inside when at least two of
its three LDNIs place it inside.

Readings where the paper is silent:
  G1  Node (i, j, k) lies at the pixel centres (c_x[i], c_y[j], c_z[k]) of
      the sampler, c[t] = f32(lo + (t + 0.5) * (hi - lo) / w) in float64.
      Its depth on the a-LDNI is f32(c_a - lo_a) (float64 difference, one
      rounding): the depth a sample exactly at the node would receive.
  G2  A node is inside according to one LDNI when the number of the ray's
      samples with depth <= the node's depth is odd.  The volumes are thus
      half-open [enter, exit): a node on an entering sample is inside, one
      on a leaving sample outside, a zero-thickness volume holds no node,
      and volumes that touch leave no gap between them.
  G3  A pixel with an odd sample count: its last, unpaired sample bounds
      nothing and is ignored (as for the Boolean operations).
  G4  The three images use the sampler's cyclic frame: the x-LDNI images
      (y, z), the y-LDNI (z, x), the z-LDNI (x, y); pixel (iu, iv) of an
      image is p = iv * w + iu.  So node (i, j, k) is on pixel k*w + j of the
      x-LDNI at depth index i, pixel i*w + k of the y-LDNI at depth index j,
      and pixel j*w + i of the z-LDNI at depth index k.
Results here are dense boolean arrays indexed [k][j][i].
"""
from __future__ import annotations

import numpy as np

from . import AxisLDNI, bbox_f32


def node_depths(lo: float, hi: float, w: int) -> np.ndarray:
    """Depths (float32) of the w nodes along one axis, measured from lo (G1)."""
    lo, hi = float(lo), float(hi)
    h = (hi - lo) / float(w)
    t = np.arange(w, dtype=np.float64)
    c = (lo + (t + 0.5) * h).astype(np.float32)
    return (c.astype(np.float64) - lo).astype(np.float32)


def node_coordinates(lo: float, hi: float, w: int) -> np.ndarray:
    """World coordinates (float32) of the w nodes along one axis (G1)."""
    lo, hi = float(lo), float(hi)
    h = (hi - lo) / float(w)
    return (lo + (np.arange(w, dtype=np.float64) + 0.5) * h).astype(np.float32)


def ray_inside(samples: np.ndarray, depths: np.ndarray) -> np.ndarray:
    """Inside flags of nodes at ``depths`` along one ray whose sorted samples
    are ``samples`` (G2, G3)."""
    paired = np.asarray(samples, dtype=np.float32)[: len(samples) // 2 * 2]
    at_or_before = np.searchsorted(paired, np.asarray(depths, dtype=np.float32), side="right")
    return at_or_before % 2 == 1


def axis_votes(ax: AxisLDNI, depths: np.ndarray) -> np.ndarray:
    """Votes of one LDNI for every node on its rays, indexed [iv][iu][t]."""
    w = ax.w
    off = ax.offsets.astype(np.int64)
    out = np.zeros((w * w, w), dtype=bool)
    for p in range(w * w):
        out[p] = ray_inside(ax.depth[off[p]:off[p + 1]], depths)
    return out.reshape(w, w, w)


def classify(x: AxisLDNI, y: AxisLDNI, z: AxisLDNI, bbox, w: int):
    """Inside/outside of all w^3 nodes.  Returns (inside, (vote_x, vote_y,
    vote_z)), each a bool array [k][j][i]."""
    for a in (x, y, z):
        if a.w != w:
            raise ValueError("the three LDNIs must have resolution w")
    b = bbox_f32(bbox)
    dx, dy, dz = (node_depths(b[a], b[3 + a], w) for a in range(3))
    vx = axis_votes(x, dx)                      # [k][j][i]
    vy = axis_votes(y, dy).transpose(1, 2, 0)   # [i][k][j] -> [k][j][i]
    vz = axis_votes(z, dz).transpose(2, 0, 1)   # [j][i][k] -> [k][j][i]
    votes = vx.astype(np.int8) + vy.astype(np.int8) + vz.astype(np.int8)
    return votes >= 2, (vx, vy, vz)


def classify_at(x: AxisLDNI, y: AxisLDNI, z: AxisLDNI, bbox, w: int, i, j, k):
    """The same classification at the listed nodes only (arrays i, j, k)."""
    b = bbox_f32(bbox)
    dx, dy, dz = (node_depths(b[a], b[3 + a], w) for a in range(3))
    i, j, k = (np.asarray(t, dtype=np.int64) for t in (i, j, k))
    out = np.zeros(i.shape, dtype=bool)

    def vote(ax, p, d):
        o0, o1 = int(ax.offsets[p]), int(ax.offsets[p + 1])
        return bool(ray_inside(ax.depth[o0:o1], [d])[0])

    for n in range(i.size):
        ii, jj, kk = int(i.flat[n]), int(j.flat[n]), int(k.flat[n])
        v = (vote(x, kk * w + jj, dx[ii]) + vote(y, ii * w + kk, dy[jj])
             + vote(z, jj * w + ii, dz[kk]))
        out.flat[n] = v >= 2
    return out


def stats(inside: np.ndarray, votes) -> tuple[int, int]:
    """(nodes inside, nodes whose three votes are not all equal)."""
    vx, vy, vz = votes
    return int(inside.sum()), int(((vx != vy) | (vy != vz)).sum())
