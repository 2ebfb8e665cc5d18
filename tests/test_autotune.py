"""The tile-shape table of the autotuner: buckets, lookups, and the shipped
table (written by ``python -m paper_1009_0794_amd.autotune`` on an MI355X)."""
import os

import pytest

from paper_1009_0794_amd import autotune


def test_bucket_rounds_resolution_and_density():
    assert autotune.bucket(512, 512 * 512) == "w512_d0"
    assert autotune.bucket(500, 4 * 500 * 500) == "w512_d2"
    assert autotune.bucket(1024, 1000) == "w1024_d-10"
    assert autotune.bucket(64, 0) == "w64_d-12"  # no triangles: the lowest density bucket


def test_lookup_exact_nearest_and_default():
    table = {"w512_d0": (8, 8), "w512_d-4": (32, 32), "w64_d3": (16, 16)}
    assert autotune.lookup(512, 512 * 512, table) == (8, 8)
    assert autotune.lookup(512, 512 * 512 // 8, table) == (32, 32)    # d-3: d-4 is nearer than d0
    assert autotune.lookup(512, 512 * 512 // 2, table) == (8, 8)      # d-1: d0 is nearer
    assert autotune.lookup(512, 512 * 512 // 16, table) == (32, 32)   # d-4 exactly
    assert autotune.lookup(2048, 10 ** 6, table) == autotune.DEFAULT   # no bucket at this resolution


def test_table_round_trip(tmp_path):
    path = os.path.join(tmp_path, "t.json")
    autotune.save_table({"w128_d1": (8, 8), "w1024_d-5": (32, 32)}, "gfx950", path)
    assert autotune.load_table(path) == {"w128_d1": (8, 8), "w1024_d-5": (32, 32)}
    assert autotune.load_table(os.path.join(tmp_path, "missing.json")) == {}


def test_shipped_table_holds_valid_shapes():
    table = autotune.load_table()
    if not table:
        pytest.skip("no tuned table in the package")
    for k, (tw, th) in table.items():
        assert k.startswith("w") and "_d" in k
        assert 8 <= tw <= 256 and 1 <= th <= 64 and tw * th <= 1024, (k, tw, th)


def test_batch_lookup_prefers_the_batch_table():
    table = {"w512_d0": (8, 8), "w512_d-4": (32, 32)}
    btable = {"w512_d0": (16, 16)}
    assert autotune.batch_lookup(512, 512 * 512, btable, table) == (16, 16)
    assert autotune.batch_lookup(512, 512 * 512 // 16, btable, table) == (32, 32)  # not in the batch table
    assert autotune.batch_lookup(2048, 10 ** 6, {}, {}) == autotune.DEFAULT


def test_shipped_batch_table_holds_valid_shapes():
    table = autotune.load_table(autotune.BATCH_TABLE_PATH)
    if not table:
        pytest.skip("no batch table in the package")
    for k, (tw, th) in table.items():
        assert k.startswith("w") and "_d" in k
        assert 8 <= tw <= 256 and 1 <= th <= 64 and tw * th <= 1024, (k, tw, th)
