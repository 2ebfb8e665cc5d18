"""TEST INFRASTRUCTURE ONLY: CPU oracle for the approximate normal sampling
of the paper (Sec. 3, "Approximate Surface Normal Sampling", with the
accuracy trade-off under "Balance between time and accuracy").

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product library shares no code with it.

The paper renders the three components of the unit normal as an RGB colour
with one byte per component, so a component c in [-1, 1] is stored with a
resolution of 256 levels.  Reading fixed here: the
colour is (c + 1) / 2 and the byte its 8-bit unsigned-normalised value rounded
to nearest, b = floor((c + 1) * 127.5 + 0.5) clamped to [0, 255], evaluated
with float64 operations in that order (exact for |c| >= 2^-29; a smaller c
rounds c + 1 to 1 and gives 128); the three bytes are packed
x | y << 8 | z << 16 in one 32-bit word; decoding maps b back to
b / 127.5 - 1.
"""
from __future__ import annotations

import numpy as np


def encode(normal) -> np.ndarray:
    """float32 [n, 3] unit normals -> uint32 [n] packed codes."""
    c = np.asarray(normal, dtype=np.float32).reshape(-1, 3).astype(np.float64)
    b = np.clip(np.floor((c + 1.0) * 127.5 + 0.5), 0.0, 255.0).astype(np.uint32)
    return b[:, 0] | (b[:, 1] << np.uint32(8)) | (b[:, 2] << np.uint32(16))


def decode(code) -> np.ndarray:
    """uint32 [n] packed codes -> float64 [n, 3] components."""
    c = np.asarray(code, dtype=np.uint32).reshape(-1)
    b = np.stack([c & 255, (c >> 8) & 255, (c >> 16) & 255], axis=1).astype(np.float64)
    return b / 127.5 - 1.0
