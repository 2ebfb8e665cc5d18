"""Host logic of bench.py (no GPU): the refusal of several GPUs, and the
counter-traffic lookup, which must go null once a kernel source no longer
matches the source its counter summary was taken from."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "paper_1009_0794_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "k.hip").write_text("kernel source, first version\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h = bench.kernel_source_hash("k.hip")
    (prof / "foo_kernel_wl_traffic.txt").write_text(
        f"# header\nkernel_source_sha256_16: {h}\nhbm_bytes_per_launch: 1.5e+09\n")
    assert bench.read_traffic("wl", "foo", "k.hip") == 1.5e9
    assert bench.read_traffic("other", "foo", "k.hip") is None  # no summary for this workload
    (src / "k.hip").write_text("kernel source, second version\n")
    assert bench.read_traffic("wl", "foo", "k.hip") is None


def test_committed_traffic_summaries_match_their_sources():
    """Every committed traffic summary names the current hash of its kernel's
    source, so bench.py reports its bytes (a kernel edited since its counters
    were taken would report null)."""
    sources = {"sample": "ldni_kernels.hip", "place": "ldni_kernels.hip", "setup": "ldni_kernels.hip",
               "bin": "ldni_kernels.hip", "backward": "ldni_backward.hip",
               "classify_nodes": "ldni_nodes.hip", "boolean_write": "ldni_boolean.hip"}
    names = [n for n in os.listdir(os.path.join(ROOT, "profiles")) if n.endswith("_traffic.txt")]
    assert names
    for n in names:
        kernel, workload = n[:-len("_traffic.txt")].split("_kernel_")
        assert bench.read_traffic(workload, kernel, sources[kernel]) is not None, n


def test_committed_atomic_summaries_match_their_sources():
    """Every committed atomics summary names the current hash of the kernel
    source, so bench.py reports the kernels' atomic rates from it."""
    names = [n for n in os.listdir(os.path.join(ROOT, "profiles")) if n.endswith("_atomics.txt")]
    assert names
    for n in names:
        workload = n[len("forward_kernels_"):-len("_atomics.txt")]
        got = bench.read_atomics(workload)
        assert got and "setup" in got, n
        assert all(v >= 0 for v in got.values())
