"""Tile-shape autotuning for the sampling kernels.

The count and write kernels run one workgroup per screen tile; the best tile
shape depends on the resolution and on how many triangles land on a pixel
(small triangles and deep pixels favour small tiles, large triangles favour
large ones).  ``tune`` times ``ldni_sample`` for each candidate shape on
the given meshes and records the fastest shape per bucket of
(resolution, triangles per pixel); ``lookup`` reads the table.  Results do
not depend on the shape, only speed does.

The table is JSON: {"arch": "...", "entries": {"w<W>_d<D>": [tw, th], ...}},
where W is the resolution rounded to a power of two and D = round(log2(T / w^2)).

Inside a batch the best shapes differ: the images share one graph and the
persistent kernels of each tile class, so ``tune_batch`` times whole batch
replays (``ldni_batch_run``) and changes one bucket's shape at a time
(coordinate descent from the plain table), writing a second table that
``sample_batch`` prefers.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, Tuple

SHAPES = [(32, 32), (16, 16), (64, 16), (32, 8), (64, 8), (128, 8), (16, 32), (8, 32), (8, 8)]
DEFAULT = (0, 0)  # the library chooses from the triangle density
HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.environ.get("LDNI_TILE_TABLE", os.path.join(HERE, "tile_table.json"))
BATCH_TABLE_PATH = os.environ.get("LDNI_BATCH_TILE_TABLE", os.path.join(HERE, "tile_table_batch.json"))


def bucket(w: int, n_tris: int) -> str:
    wb = 1 << max(0, int(round(math.log2(max(1, w)))))
    d = n_tris / float(max(1, w * w))
    db = int(round(math.log2(max(d, 2.0 ** -12))))
    return f"w{wb}_d{db}"


def load_table(path: str = TABLE_PATH) -> Dict[str, Tuple[int, int]]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        doc = json.load(f)
    return {k: tuple(v) for k, v in doc.get("entries", {}).items()}


def save_table(entries: Dict[str, Tuple[int, int]], arch: str, path: str = TABLE_PATH) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"arch": arch, "entries": {k: list(v) for k, v in sorted(entries.items())}}, f, indent=1)
    os.replace(tmp, path)


def lookup(w: int, n_tris: int, table=None) -> Tuple[int, int]:
    """Tile shape for a mesh of n_tris triangles sampled at w (the nearest
    tuned density bucket at the same resolution, else the default)."""
    table = load_table() if table is None else table
    k = bucket(w, n_tris)
    if k in table:
        return table[k]
    wkey = k.split("_")[0]
    d = int(k.split("_d")[1])
    near = [(abs(int(kk.split("_d")[1]) - d), kk) for kk in table if kk.startswith(wkey + "_")]
    return table[min(near)[1]] if near else DEFAULT


def time_shape(ldni, torch, verts, tris, bbox, w, shape, reps=5) -> float:
    """Mean milliseconds of one 3-axis ldni_sample with the given tile shape."""
    ldni.set_tile_shape(*shape)
    for _ in range(2):
        ldni.ldni_sample(verts, tris, bbox, w, "xyz").free()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        ldni.ldni_sample(verts, tris, bbox, w, "xyz").free()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(meshes: Iterable, shapes=SHAPES, reps=5, table=None, verbose=False) -> Dict[str, Tuple[int, int]]:
    """Time every shape on every mesh ((verts, tris, bbox, w) with device
    tensors) and keep, per bucket, the shape with the least total time."""
    import torch

    import paper_1009_0794_amd as ldni
    table = dict(load_table() if table is None else table)
    totals: Dict[str, Dict[Tuple[int, int], float]] = {}
    for verts, tris, bbox, w in meshes:
        k = bucket(w, int(tris.shape[0]))
        for sh in shapes:
            ms = time_shape(ldni, torch, verts, tris, bbox, w, sh, reps)
            totals.setdefault(k, {}).setdefault(sh, 0.0)
            totals[k][sh] += ms
            if verbose:
                print(f"{k} tile {sh[0]}x{sh[1]}: {ms:.3f} ms", flush=True)
    ldni.set_tile_shape(*DEFAULT)
    for k, per in totals.items():
        table[k] = min(per.items(), key=lambda kv: kv[1])[0]
    return table


def batch_lookup(w: int, n_tris: int, batch_table=None, table=None) -> Tuple[int, int]:
    """Tile shape for a mesh inside a batch: the batch table's bucket if it
    has one, else ``lookup``."""
    batch_table = load_table(BATCH_TABLE_PATH) if batch_table is None else batch_table
    k = bucket(w, n_tris)
    if k in batch_table:
        return batch_table[k]
    return lookup(w, n_tris, table)


def time_batch(ldni, torch, meshes, shapes, reps=3) -> float:
    """Mean milliseconds of one replay of the batch of meshes ((verts, tris,
    bbox, w) with device tensors), mesh k sampled with tile shape shapes[k]."""
    b = ldni.sample_batch([(v, t, bb, w, sh) for (v, t, bb, w), sh in zip(meshes, shapes)], "xyz", tiles=None)
    try:
        b.run()
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            b.run()
        e.record()
        torch.cuda.synchronize()
        return a.elapsed_time(e) / reps
    finally:
        b.free()


def tune_batch(meshes, shapes=SHAPES, reps=4, table=None, rounds=1, top=16, gain=0.995,
               verbose=False) -> Dict[str, Tuple[int, int]]:
    """Coordinate descent over the buckets of one batch: start from the plain
    table's shapes and, bucket by bucket (the `top` buckets with the most
    work, triangles plus pixels of three images, first), keep a shape whose
    batch replay is faster by more than the noise (below `gain` times the
    best so far).  Returns the buckets' shapes (the batch table)."""
    import torch

    import paper_1009_0794_amd as ldni
    table = dict(load_table() if table is None else table)
    keys = [bucket(w, int(t.shape[0])) for _, t, _, w in meshes]
    cur = {k: tuple(lookup(w, int(t.shape[0]), table)) for k, (_, t, _, w) in zip(keys, meshes)}
    weight: Dict[str, int] = {}
    for k, (_, t, _, w) in zip(keys, meshes):
        weight[k] = weight.get(k, 0) + int(t.shape[0]) + 3 * w * w
    order = sorted(weight, key=lambda k: -weight[k])[:top]
    best = time_batch(ldni, torch, meshes, [cur[k] for k in keys], reps)
    if verbose:
        print(f"start: {best:.3f} ms", flush=True)
    for _ in range(rounds):
        for k in order:
            for sh in shapes:
                if sh == cur[k]:
                    continue
                trial = dict(cur)
                trial[k] = sh
                ms = time_batch(ldni, torch, meshes, [trial[q] for q in keys], reps)
                if verbose:
                    print(f"{k} tile {sh[0]}x{sh[1]}: {ms:.3f} ms (best {best:.3f})", flush=True)
                if ms < gain * best:
                    best, cur = ms, trial
    return cur


if __name__ == "__main__":
    # Tune on the seeded batch workload and the single-mesh workloads, then
    # write the table next to this file (or to $LDNI_TILE_TABLE).
    import sys

    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1009_0794_amd import meshgen as mg

    if "--batch" in sys.argv:
        # the batch table, tuned on the seeded 256-mesh batch itself
        ms = mg.c4_batch256()
        meshes = [(torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.tris).cuda(), m.bbox, m.w) for m in ms]
        btable = tune_batch(meshes, verbose=True)
        save_table(btable, torch.cuda.get_device_properties(0).gcnArchName, BATCH_TABLE_PATH)
        print(json.dumps({k: list(v) for k, v in sorted(btable.items())}))
        sys.exit(0)
    meshes = []
    pool = mg.c4_batch256(n=48) + [mg.c2_flower(), mg.c1_icosphere()]
    seen = set()
    for m in pool:
        k = bucket(m.w, m.n_tris)
        if k in seen:
            continue
        seen.add(k)
        meshes.append((torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.tris).cuda(), m.bbox, m.w))
    table = tune(meshes, verbose=True)
    arch = torch.cuda.get_device_properties(0).gcnArchName
    save_table(table, arch)
    print(json.dumps({k: list(v) for k, v in sorted(table.items())}))
