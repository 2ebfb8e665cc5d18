"""Write the exact-arithmetic LDNI fixtures in this folder.

The expected values come only from ``oracle.exact`` (rational arithmetic on
the ray-casting definition, Sec. 2 Definitions 1-2) on tiny adversarial
meshes whose vertices, edges and faces sit exactly on pixel-centre rays, so
that the tie rule for rays through edges and vertices (Remark 1; Definition 4)
is exercised on every axis.  Run from the repository root:

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402
from tests.golden.fixture_meshes import FIXTURES  # noqa: E402


def main():
    for name, (verts, tris, bbox, w) in FIXTURES.items():
        res = exact.sample(verts, tris, bbox, w)
        doc = {
            "name": name,
            "source": "oracle.exact (rational evaluation of Sec. 2 Definitions 1-2, tie rule of Remark 1)",
            "bbox": [float(x) for x in bbox],
            "w": int(w),
            "verts": np.asarray(verts, np.float32).astype(float).tolist(),
            "tris": np.asarray(tris, np.int64).tolist(),
            "axes": {},
        }
        for a, pix in res.items():
            doc["axes"]["xyz"[a]] = [[[f"{d.numerator}/{d.denominator}", int(t)] for d, t in hits]
                                      for hits in pix]
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(doc, f, separators=(",", ":"))
        print(name, {k: sum(len(p) for p in v) for k, v in doc["axes"].items()})


if __name__ == "__main__":
    main()
