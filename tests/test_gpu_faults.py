"""Failure handling forced from the host: with LDNI_FAULT=alloc every device
allocation the library makes fails as if the device were out of memory.
Each entry point must return LDNI_ERR_OUT_OF_MEMORY (no output, nothing
launched that reads unallocated memory), and a call made after the fault
is lifted must work and match the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1009_0794_amd as ldni
from paper_1009_0794_amd import meshgen as mg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
OOM = 3


def _mesh():
    m = mg.c1_icosphere()
    return m, torch.from_numpy(m.verts).to(DEV), torch.from_numpy(m.tris).to(DEV)


def test_allocation_failure_is_reported_and_recovered(monkeypatch):
    m, v, f = _mesh()
    good = ldni.sample(v, f, m.bbox, 64, "xyz")  # inputs for the derived operations
    torch.cuda.synchronize()
    # buffers cached from earlier calls would satisfy requests without an
    # allocation: hand them back first
    ldni.ldni_trim()
    monkeypatch.setenv("LDNI_FAULT", "alloc")
    calls = {
        "ldni_sample": lambda: ldni.ldni_sample(v, f, m.bbox, 64, "xyz"),
        "ldni_sample_begin": lambda: ldni.sample(v, f, m.bbox, 64, "xyz"),
        "ldni_batch_create": lambda: ldni.sample_batch([(v, f, m.bbox, 64)], "xyz"),
        "ldni_boolean": lambda: ldni.ldni_boolean(good[2], good[2], "union"),
        "ldni_offset": lambda: ldni.ldni_offset(good, m.bbox, 0.05),
        "ldni_classify_nodes": lambda: ldni.classify_nodes(good, m.bbox),
    }
    for name, call in calls.items():
        with pytest.raises(ldni.LDNIError) as e:
            call()
        assert e.value.code == OOM, f"{name}: {e.value}"
    monkeypatch.delenv("LDNI_FAULT")
    # a good call afterwards
    got = ldni.sample(v, f, m.bbox, 64, "xyz")
    torch.cuda.synchronize()
    ref = oracle.sample(m.verts, m.tris, m.bbox, 64)
    for a in range(3):
        assert np.array_equal(got[a].offsets.cpu().numpy().view(np.uint32), ref[a].offsets)
        assert np.array_equal(got[a].tri.cpu().numpy(), ref[a].tri)
        assert np.array_equal(got[a].depth.cpu().numpy().view(np.uint32), ref[a].depth.view(np.uint32))
    b = ldni.sample_batch([(v, f, m.bbox, 64)], "xyz")
    for a in range(3):
        assert torch.equal(b.to_torch(0, a).depth, got[a].depth)
    b.free()
