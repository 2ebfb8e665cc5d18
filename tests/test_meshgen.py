"""The seeded synthetic inputs: sizes, closedness, outward orientation."""
import numpy as np
import pytest

from paper_1009_0794_amd import meshgen as mg
from tests.meshcheck import is_closed_oriented, volume
from tests.golden.fixture_meshes import FIXTURES


def test_icosphere_counts():
    for lvl in range(5):
        v, f = mg.icosphere(lvl)
        assert len(v) == 10 * 4 ** lvl + 2 and len(f) == 20 * 4 ** lvl
        assert is_closed_oriented(f)
        assert volume(v, f) > 0


def test_c1():
    m = mg.c1_icosphere()
    assert (m.n_verts, m.n_tris, m.w) == (642, 1280, 128)
    assert m.verts.dtype == np.float32 and m.tris.dtype == np.int32
    assert is_closed_oriented(m.tris)
    assert 0.95 * 4 / 3 * np.pi < volume(m.verts, m.tris) < 4 / 3 * np.pi


def test_c2_flower():
    m = mg.c2_flower()
    assert (m.n_verts, m.n_tris, m.w) == (130562, 261120, 512)
    assert is_closed_oriented(m.tris)
    assert volume(m.verts, m.tris) > 0
    r = np.linalg.norm(m.verts.astype(np.float64), axis=1)
    assert r.max() < 1.4 and r.min() > 0.6
    # seeded: the same call gives the same bits
    assert np.array_equal(m.verts, mg.c2_flower().verts)


def test_small_solids():
    for v, f in (mg.box_mesh((0, 0, 0), (1, 2, 3)), mg.octahedron(),
                 mg.torus(16, 8, 1.0, 0.3), mg.uv_flower(8, 16, np.random.default_rng(0))):
        assert is_closed_oriented(f)
        assert volume(v, f) > 0
    assert abs(volume(*mg.box_mesh((0, 0, 0), (1, 2, 3))) - 6.0) < 1e-12


def test_fixtures_closed():
    for name, (v, f, bb, w) in FIXTURES.items():
        assert is_closed_oriented(f), name
        assert volume(v, f) > 0, name


@pytest.mark.slow
def test_c3_scene64():
    m = mg.c3_scene64()
    assert m.n_tris == 2152448 and m.w == 2048
    assert is_closed_oriented(m.tris)
    assert np.abs(m.verts).max() < 1.1


def test_c4_batch_shapes():
    ms = mg.c4_batch256(n=12)
    assert len(ms) == 12
    for m in ms:
        assert m.w in (64, 128, 256, 512, 1024)
        assert is_closed_oriented(m.tris)
        assert volume(m.verts, m.tris) > 0
        bb = np.array(m.bbox)
        assert (m.verts >= bb[:3]).all() and (m.verts <= bb[3:]).all()
