"""Pins of the 8-bit normal codec oracle (Sec. 3, approximate surface normal
sampling): closed-form levels, the quantisation bound, monotonicity, and an
exact rational evaluation of the rounding."""
from fractions import Fraction

import numpy as np

from oracle import normal_codec as nc


def test_levels_of_the_extremes_and_zero():
    n = np.array([[-1, 0, 1], [1, -1, 0], [0, 0, 0]], np.float32)
    codes = nc.encode(n)
    assert list(codes) == [0 | 128 << 8 | 255 << 16, 255 | 0 << 8 | 128 << 16, 128 | 128 << 8 | 128 << 16]
    assert (codes >> 24 == 0).all()


def test_within_half_a_step_of_random_unit_normals():
    rng = np.random.default_rng(0)
    n = rng.normal(size=(20000, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    err = np.abs(nc.decode(nc.encode(n)) - n.astype(np.float64))
    assert err.max() <= 1.0 / 255.0 + 1e-12  # 256 levels on [-1, 1]: half of 2/255
    assert err.max() > 0.9 / 255.0


def test_monotone_and_every_level_used():
    c = np.linspace(-1.0, 1.0, 100001).astype(np.float32)
    b = nc.encode(np.stack([c, c, c], axis=1)) & 255
    assert (np.diff(b.astype(np.int64)) >= 0).all()
    assert set(b.tolist()) == set(range(256))


def test_matches_exact_rational_rounding():
    """For |c| >= 2^-29 every float64 step is exact, so the byte is the exact
    rational rounding; smaller components round c + 1 to 1 (byte 128)."""
    rng = np.random.default_rng(1)
    c = np.concatenate([rng.uniform(-1, 1, 3000),
                        # exact midpoints between levels and their float32 neighbours
                        (np.arange(256) + 0.5) / 127.5 - 1.0]).astype(np.float32)
    c = np.concatenate([c, np.nextafter(c, np.float32(2)), np.nextafter(c, np.float32(-2))])
    c = np.clip(c, -1, 1).astype(np.float32)
    got = nc.encode(np.stack([c, c, c], axis=1)) & 255
    for x, g in zip(c.tolist(), got.tolist()):
        if abs(x) >= 2.0 ** -29:
            want = ((Fraction(x) + 1) * Fraction(255, 2) + Fraction(1, 2)).__floor__()
            assert g == min(max(int(want), 0), 255), x
        else:
            assert g == 128, x


def test_components_beyond_the_unit_range_clamp():
    """The reading clamps the byte to [0, 255]: components a little beyond
    +-1 (a normal that is not quite unit length) still give 255 and 0, and so
    do components far outside."""
    c = np.array([1.0, 1.003, 1.004, 1.5, 7.0, -1.0, -1.004, -1.5, -7.0], np.float32)
    got = nc.encode(np.stack([c, c, c], axis=1)) & 255
    assert got.tolist() == [255, 255, 255, 255, 255, 0, 0, 0, 0]
