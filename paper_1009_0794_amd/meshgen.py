"""Seeded synthetic closed triangle meshes used as sampling inputs.

The paper's own models (octa-flower, dragon, gear, bunny, Beethoven; Sec. 6,
Tables 2-4) are not available, so these generators build stand-ins with the
same structure: star-shaped "petal" solids like the octa-flower of Fig. 1,
nested shells with high depth complexity like the dragon's 14 layers
(Table 2), and mixed-size batches.

Every mesh is a closed, 2-manifold, counter-clockwise-outward triangle mesh
(every edge used twice in opposite directions, positive enclosed volume), the
input contract of Sec. 2 (Remark 2) and Sec. 3.  Vertices are float32 ``[V,3]``,
triangles int32 ``[T,3]``; a bounding box is ``(xlo, ylo, zlo, xhi, yhi, zhi)``.

This module only builds geometry: it performs none of the sampling
arithmetic, and is shared by the tests, the oracle checks and the benchmark.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Mesh", "icosphere", "uv_flower", "torus", "concat", "random_rotation",
    "c1_icosphere", "c2_flower", "c3_scene64", "c4_batch256", "c5_target",
    "box_mesh", "octahedron", "cubic_bbox",
]


@dataclass
class Mesh:
    verts: np.ndarray          # float32 [V,3]
    tris: np.ndarray           # int32 [T,3]
    bbox: tuple                # (xlo, ylo, zlo, xhi, yhi, zhi)
    w: int = 0                 # sampling resolution this mesh is meant for
    name: str = ""

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


# --------------------------------------------------------------------------
# primitive shells (computed in float64, returned as float64; callers cast)
# --------------------------------------------------------------------------

def _icosahedron():
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    # cyclic permutations of (0, +-1, +-phi)
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((0.0, s1, s2 * phi))
            v.append((s1, s2 * phi, 0.0))
            v.append((s2 * phi, 0.0, s1))
    v = np.array(v, dtype=np.float64)
    faces = []
    n = len(v)
    for a in range(n):
        for b in range(a + 1, n):
            if abs(np.linalg.norm(v[a] - v[b]) - 2.0) > 1e-9:
                continue
            for c in range(b + 1, n):
                if (abs(np.linalg.norm(v[a] - v[c]) - 2.0) < 1e-9
                        and abs(np.linalg.norm(v[b] - v[c]) - 2.0) < 1e-9):
                    nrm = np.cross(v[b] - v[a], v[c] - v[a])
                    if np.dot(nrm, v[a] + v[b] + v[c]) < 0:
                        faces.append((a, c, b))
                    else:
                        faces.append((a, b, c))
    assert len(faces) == 20
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, np.array(faces, dtype=np.int64)


def _icosphere64(level: int):
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}
        nf = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = (np.asarray(verts[a]) + np.asarray(verts[b])) * 0.5
                m = m / np.linalg.norm(m)
                idx = len(verts)
                verts.append(tuple(m))
                cache[key] = idx
            return idx

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    return np.array(verts, dtype=np.float64), f


_ICO_CACHE: dict = {}


def icosphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0), rot=None):
    """Unit icosahedron subdivided ``level`` times (edge midpoints pushed to
    the sphere in float64): V = 10*4^L + 2, T = 20*4^L."""
    if level not in _ICO_CACHE:
        _ICO_CACHE[level] = _icosphere64(level)
    v, f = _ICO_CACHE[level]
    v = v.copy()
    if rot is not None:
        v = v @ np.asarray(rot).T
    v = v * radius + np.asarray(center, dtype=np.float64)
    return v, f.copy()


def uv_flower(n_theta: int, n_phi: int, rng=None, sigma: float = 0.01,
              amp: float = 0.3, petals: int = 8):
    """UV sphere with radius r = 1 + amp*cos(petals*phi)*sin(theta)^2 + N(0,sigma)
    per vertex (poles included), a star-shaped 'octa-flower' stand-in.
    V = 2 + (n_theta-1)*n_phi, T = 2*n_phi*(n_theta-1)."""
    nr = n_theta - 1
    th = math.pi * np.arange(1, n_theta) / n_theta
    ph = 2.0 * math.pi * np.arange(n_phi) / n_phi
    TH, PH = np.meshgrid(th, ph, indexing="ij")          # [nr, n_phi]
    theta = np.concatenate([[0.0], TH.ravel(), [math.pi]])
    phi = np.concatenate([[0.0], PH.ravel(), [0.0]])
    r = 1.0 + amp * np.cos(petals * phi) * np.sin(theta) ** 2
    if rng is not None and sigma > 0:
        r = r + rng.normal(0.0, sigma, size=r.shape)
    v = np.stack([r * np.sin(theta) * np.cos(phi),
                  r * np.sin(theta) * np.sin(phi),
                  r * np.cos(theta)], axis=1)
    v[0] = (0.0, 0.0, r[0])
    v[-1] = (0.0, 0.0, -r[-1])
    north, south = 0, 1 + nr * n_phi
    ring = lambda j, i: 1 + j * n_phi + (i % n_phi)
    f = []
    i = np.arange(n_phi)
    f.append(np.stack([np.full(n_phi, north), ring(0, i), ring(0, i + 1)], 1))
    for j in range(nr - 1):
        a, b = ring(j, i), ring(j, i + 1)
        c, d = ring(j + 1, i), ring(j + 1, i + 1)
        f.append(np.stack([a, c, d], 1))
        f.append(np.stack([a, d, b], 1))
    f.append(np.stack([np.full(n_phi, south), ring(nr - 1, i + 1), ring(nr - 1, i)], 1))
    return v, np.concatenate(f).astype(np.int64)


def torus(n_u: int, n_v: int, R: float, r: float, center=(0.0, 0.0, 0.0), rot=None):
    """Ring torus with n_u segments around the major circle and n_v around
    the tube: T = 2*n_u*n_v."""
    u = 2.0 * math.pi * np.arange(n_u) / n_u
    v = 2.0 * math.pi * np.arange(n_v) / n_v
    U, Vv = np.meshgrid(u, v, indexing="ij")
    x = (R + r * np.cos(Vv)) * np.cos(U)
    y = (R + r * np.cos(Vv)) * np.sin(U)
    z = r * np.sin(Vv)
    verts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    idx = lambda a, b: (a % n_u) * n_v + (b % n_v)
    A, B = np.meshgrid(np.arange(n_u), np.arange(n_v), indexing="ij")
    A, B = A.ravel(), B.ravel()
    p00, p10, p01, p11 = idx(A, B), idx(A + 1, B), idx(A, B + 1), idx(A + 1, B + 1)
    f = np.concatenate([np.stack([p00, p10, p11], 1), np.stack([p00, p11, p01], 1)])
    # orient outward: enclosed volume must be positive
    if _volume64(verts, f) < 0:
        f = f[:, [0, 2, 1]]
    if rot is not None:
        verts = verts @ np.asarray(rot).T
    verts = verts + np.asarray(center, dtype=np.float64)
    return verts, f.astype(np.int64)


def _volume64(v, f):
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def random_rotation(rng) -> np.ndarray:
    """Uniform random rotation from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def concat(parts):
    """Concatenate (verts64, tris) shells into one float32/int32 mesh."""
    vs, fs, off = [], [], 0
    for v, f in parts:
        vs.append(v)
        fs.append(f + off)
        off += len(v)
    return (np.ascontiguousarray(np.concatenate(vs).astype(np.float32)),
            np.ascontiguousarray(np.concatenate(fs).astype(np.int32)))


def cubic_bbox(verts, pad: float = 0.05):
    """The mesh AABB made cubic (longest side) and padded by ``pad`` of it."""
    lo = verts.min(0).astype(np.float64)
    hi = verts.max(0).astype(np.float64)
    c = 0.5 * (lo + hi)
    half = 0.5 * float((hi - lo).max()) * (1.0 + pad)
    if half <= 0:
        half = 1.0
    return tuple(float(x) for x in np.concatenate([c - half, c + half]))


# --------------------------------------------------------------------------
# small closed test solids
# --------------------------------------------------------------------------

def box_mesh(lo, hi):
    """Axis-aligned box [lo,hi] as 12 outward triangles (8 vertices)."""
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]],
                 dtype=np.float64)
    f = np.array([[0, 2, 1], [0, 3, 2],      # z = z0, normal -z
                  [4, 5, 6], [4, 6, 7],      # z = z1, normal +z
                  [0, 1, 5], [0, 5, 4],      # y = y0, normal -y
                  [3, 7, 6], [3, 6, 2],      # y = y1, normal +y
                  [0, 4, 7], [0, 7, 3],      # x = x0, normal -x
                  [1, 2, 6], [1, 6, 5]],     # x = x1, normal +x
                 dtype=np.int64)
    return v, f


def octahedron(center=(0.0, 0.0, 0.0), radius=1.0):
    c = np.asarray(center, dtype=np.float64)
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64) * radius + c
    f = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4],
                  [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]], dtype=np.int64)
    return v, f


# --------------------------------------------------------------------------
# the five benchmark workloads
# --------------------------------------------------------------------------

def c1_icosphere() -> Mesh:
    """Icosphere radius 1, level 3 (642 V, 1,280 T), bbox [-1.1,1.1]^3, w=128."""
    v, f = icosphere(3)
    v, f = concat([(v, f)])
    return Mesh(v, f, (-1.1, -1.1, -1.1, 1.1, 1.1, 1.1), 128, "icosphere-L3")


def c2_flower(seed: int = 0, n_theta: int = 256, n_phi: int = 512, w: int = 512) -> Mesh:
    """Seeded flower: UV sphere 512x256 (130,562 V, 261,120 T) with
    r = 1 + 0.3 cos(8 phi) sin^2(theta) + N(0, 0.01), bbox [-1.4,1.4]^3."""
    rng = np.random.default_rng(seed)
    v, f = uv_flower(n_theta, n_phi, rng)
    v, f = concat([(v, f)])
    return Mesh(v, f, (-1.4, -1.4, -1.4, 1.4, 1.4, 1.4), w, "flower-512x256")


def c5_target(base: Mesh, seed: int = 3, sigma: float = 0.005) -> Mesh:
    """Perturbed copy of a mesh: same topology, each vertex moved radially by
    an extra N(0, sigma)."""
    rng = np.random.default_rng(seed)
    v = base.verts.astype(np.float64)
    nrm = np.linalg.norm(v, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    v = v + rng.normal(0.0, sigma, size=(len(v), 1)) * v / nrm
    return Mesh(np.ascontiguousarray(v.astype(np.float32)), base.tris.copy(), base.bbox,
                base.w, base.name + "-perturbed")


def c3_scene64(seed: int = 1, w: int = 2048) -> Mesh:
    """64 disjoint closed shells in [-1.1,1.1]^3 (2,152,448 T), up to 32 layers.

    The domain is a 4x4x4 lattice of 0.55-wide cells.  A nest of 16
    concentric icospheres (r = 0.45 - 0.025k) sits at the origin; the 32 cells
    with at most one central index hold 16 tori and 16 icospheres; 16 of the
    24 cells with exactly two central indices hold a small icosphere at the
    corner farthest from the nest axis."""
    rng = np.random.default_rng(seed)
    parts = []
    for k in range(16):
        lvl = 6 if k < 4 else (5 if k < 10 else 4)
        parts.append(icosphere(lvl, 0.45 - 0.025 * k, (0, 0, 0), random_rotation(rng)))
    cell = 0.55
    ctr = lambda i: -1.1 + cell * (i + 0.5)
    central = lambda i: i in (1, 2)
    outer, shadow = [], []
    for a in range(4):
        for b in range(4):
            for c in range(4):
                n = int(central(a)) + int(central(b)) + int(central(c))
                if n <= 1:
                    outer.append((a, b, c))
                elif n == 2:
                    shadow.append((a, b, c))
    assert len(outer) == 32 and len(shadow) == 24
    kinds = np.array(["torus"] * 16 + ["ico6"] * 8 + ["ico5"] * 8)
    rng.shuffle(kinds)
    for (a, b, c), kind in zip(outer, kinds):
        cen = (ctr(a), ctr(b), ctr(c))
        rot = random_rotation(rng)
        if kind == "torus":
            while True:
                R = rng.uniform(0.1, 0.3)
                r = rng.uniform(0.02, 0.08)
                if R + r <= 0.27:
                    break
            parts.append(torus(256, 64, R, r, cen, rot))
        else:
            rad = rng.uniform(0.1, 0.25)
            parts.append(icosphere(6 if kind == "ico6" else 5, rad, cen, rot))
    chosen = rng.choice(len(shadow), size=16, replace=False)
    for k in sorted(chosen):
        a, b, c = shadow[k]
        idx = (a, b, c)
        rad = rng.uniform(0.05, 0.1)
        cen = []
        for d in range(3):
            lo_d = -1.1 + cell * idx[d]
            if central(idx[d]):
                # push toward the cell face farthest from the origin axis
                far = lo_d if idx[d] == 1 else lo_d + cell
                inward = 1.0 if idx[d] == 1 else -1.0
                cen.append(far + inward * (rad + 0.01))
            else:
                cen.append(lo_d + 0.5 * cell)
        parts.append(icosphere(5, rad, tuple(cen), random_rotation(rng)))
    v, f = concat(parts)
    return Mesh(v, f, (-1.1, -1.1, -1.1, 1.1, 1.1, 1.1), w, "scene64")


def c4_batch256(seed: int = 2, n: int = 256, t_lo: float = 1e3, t_hi: float = 5e5):
    """256 seeded meshes (flower / torus / icosphere), target triangle counts
    log-uniform in [1e3, 5e5], each with its own w in {64,...,1024} and a cubic
    bbox padded by 5%."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(n):
        kind = ("flower", "torus", "icosphere")[rng.integers(0, 3)]
        tstar = math.exp(rng.uniform(math.log(t_lo), math.log(t_hi)))
        w = int((64, 128, 256, 512, 1024)[rng.integers(0, 5)])
        if kind == "icosphere":
            lvl = int(min(7, max(3, round(math.log(tstar / 20.0, 4)))))
            v, f = icosphere(lvl, 1.0, (0, 0, 0), random_rotation(rng))
        elif kind == "flower":
            nt = max(4, int(round(math.sqrt(tstar / 4.0))))
            sub = np.random.default_rng([seed, m])
            v, f = uv_flower(nt, 2 * nt, sub)
        else:
            nv = max(3, int(round(math.sqrt(tstar / 4.0))))
            r = rng.uniform(0.2, 0.5)
            v, f = torus(2 * nv, nv, 1.0, r, (0, 0, 0), random_rotation(rng))
        vv, ff = concat([(v, f)])
        out.append(Mesh(vv, ff, cubic_bbox(vv), w, f"{kind}-{len(ff)}"))
    return out
