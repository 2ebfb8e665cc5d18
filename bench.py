#!/usr/bin/env python3
"""Throughput of LDNI sampling on one MI355X.

Headline step: one pass of the sampling path (triangle setup, tile binning,
sampling pass, scans, place pass with the per-pixel sort, all three axes)
over the scene64 mesh
(2,152,448 triangles, w=2048) through the C ABI call ``ldni_sample``
(library-owned outputs from the stream-ordered pool) followed by
``ldni_free``.  Inputs are resident in HBM before the timed region starts.
The metric is LDNI samples written per second, summed over the three axes.

The same JSON line also carries the metric's other parts: the flower at
w=512, the batched path (256 meshes in one captured graph vs 256 plain
calls) and forward + backward on the flower.  ``--workload`` picks a single
part (used for profiling runs).

Prints ONE JSON line.  ``--gpus`` above 1 is refused: this sampler runs on
one GPU (how it would shard is described with the design).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64 (256 CUs x 2.4 GHz x 64 lanes x 2 flops per FMA)
# algorithmic arithmetic of the sampling pass: per candidate pixel the exact
# coverage test (6 translations into the ray frame, 3 edge functions of one
# product and one fused multiply-add); per hit the barycentric depth
# (2 adds for the denominator, 5 for the numerator, divide, add, subtract)
FLOPS_PER_CANDIDATE = 15
FLOPS_PER_HIT = 10
METRIC = "LDNI samples written/sec (3 axes) at w=512/2048; batched vs plain; fwd+bwd"

PLAIN = {
    "scene64-2048": ("c3_scene64", "64 disjoint closed shells, 2,152,448 triangles, up to 32 layers, "
                                   "w=2048, 3 axes"),
    "flower-512": ("c2_flower", "seeded flower UV sphere 512x256, 261,120 triangles, w=512, 3 axes"),
    "icosphere-128": ("c1_icosphere", "icosphere level 3, 1,280 triangles, w=128, 3 axes"),
}


def kernel_source_hash(source: str = "ldni_kernels.hip") -> str:
    p = os.path.join(ROOT, "paper_1009_0794_amd", "csrc", source)
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def read_traffic(workload: str, kernel: str, source: str = "ldni_kernels.hip"):
    """HBM bytes per launch of ``kernel`` (defined in ``source``) from the
    committed counter summary, or None if there is none or the kernel source
    changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_kernel_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_source_hash(source):
        return None
    m = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def read_atomics(workload: str, source: str = "ldni_kernels.hip"):
    """Global atomic requests per launch of each forward kernel, from the
    committed counter summary ({} if there is none or the source changed)."""
    path = os.path.join(ROOT, "profiles", f"forward_kernels_{workload}_atomics.txt")
    if not os.path.exists(path):
        return {}
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_source_hash(source):
        return {}
    return {k: float(v) for k, v in re.findall(r"^(\w+): requests_per_launch ([0-9.eE+]+)", txt, re.M)}


def atomic_probe(torch, n: int = 1 << 21, words: int = 49152, reps: int = 10):
    """Float atomic adds at random addresses (torch's index_add_, one atomic
    per element): the global atomic rate a plain kernel reaches on this GPU,
    the ceiling the kernels' atomic rates are compared with."""
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    idx = torch.randint(0, words, (n,), device="cuda", generator=g)
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.zeros(words, dtype=torch.float32, device="cuda")
    dst.index_add_(0, idx, src)
    with Timer(torch) as t:
        for _ in range(reps):
            dst.index_add_(0, idx, src)
    return {"atomics_per_call": n, "G_per_s": round(n * reps / (t.ms / 1e3) / 1e9, 2),
            "how": f"index_add_ of {n} float32 values at random indices of {words} words"}


def fwd_bytes(mesh, samples):
    """Algorithmic bytes of one 3-axis forward: read the mesh once, write the
    offsets and the (depth, normal) samples once."""
    return 12 * mesh.n_verts + 12 * mesh.n_tris + 3 * 4 * (mesh.w * mesh.w + 1) + 16 * samples


def kernel_alg_bytes(name, mesh, samples):
    """The share of the algorithmic bytes each kernel moves (per step)."""
    return {"setup": 12 * mesh.n_verts + 12 * mesh.n_tris,
            "scan_pixels": 3 * 4 * (mesh.w * mesh.w + 1),
            "place": 16 * samples}.get(name)


def candidate_count(mesh, axes=(0, 1, 2)) -> int:
    """Candidate pixels of the sampling pass: for every triangle and axis, the
    pixels of its rectangle (centres c with min <= c < max in both image
    coordinates, centres rounded to float32 as the sampler does)."""
    lo = np.asarray(mesh.bbox[:3], np.float64)
    hi = np.asarray(mesh.bbox[3:], np.float64)
    P = mesh.verts[mesh.tris]  # (T, 3, 3) float32
    total = 0
    for a in axes:
        ext = []
        for d in ((a + 1) % 3, (a + 2) % 3):
            h = (hi[d] - lo[d]) / mesh.w
            c = (lo[d] + (np.arange(mesh.w, dtype=np.float64) + 0.5) * h).astype(np.float32)
            mn = P[:, :, d].min(axis=1)
            mx = P[:, :, d].max(axis=1)
            ext.append(np.searchsorted(c, mx, "left").astype(np.int64)
                       - np.searchsorted(c, mn, "left").astype(np.int64))
        total += int((np.maximum(ext[0], 0) * np.maximum(ext[1], 0)).sum())
    return total


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads() -> int:
    threads = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        threads = min(threads, int(env))
    return threads


def cpu_baseline(mesh, seconds: float):
    """The oracle on the same workload, all three axes, repeated until about
    ``seconds`` of CPU work, on the host's threads; its mean rate.  Also the
    oracle on one thread over a band of rows (the same per-pixel work, so
    its rate per sample carries over)."""
    import oracle
    threads = oracle_threads()
    samples, passes = 0, 0
    t0 = time.perf_counter()
    while True:
        r = oracle.sample(mesh.verts, mesh.tris, mesh.bbox, mesh.w, axes="xyz", nthreads=threads)
        samples += sum(r[a].n for a in range(3))
        passes += 1
        del r
        elapsed = time.perf_counter() - t0
        if elapsed >= seconds or passes >= 20:
            break
    # single thread: rows [w/2 - w/16, w/2 + w/16) of every axis (through the
    # densest part of the scene)
    j0, j1 = mesh.w // 2 - mesh.w // 16, mesh.w // 2 + mesh.w // 16
    t1 = time.perf_counter()
    r1 = oracle.sample(mesh.verts, mesh.tris, mesh.bbox, mesh.w, axes="xyz", nthreads=1,
                       window=(0, mesh.w, j0, j1))
    one = sum(r1[a].n for a in range(3))
    el1 = time.perf_counter() - t1
    return {"value": samples / elapsed, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"the whole workload (3 axes, culled mode) {passes} time(s): "
                      f"{samples} samples in {elapsed:.1f} s on {threads} threads",
            "single_thread": {"value": one / el1, "unit": "samples/s",
                              "sample": f"rows [{j0}, {j1}) of each axis, culled mode: {one} samples "
                                        f"in {el1:.1f} s"}}


def oracle_c1_seconds():
    """The C1 icosphere (w = 128, 3 axes) on the oracle: the literal
    brute-force mode (every pixel x every triangle) and the culled mode, one
    thread and all threads."""
    import oracle
    from paper_1009_0794_amd import meshgen as mg
    m = mg.c1_icosphere()
    out = {}
    for mode, brute in (("brute", True), ("culled", False)):
        for nt in (1, oracle_threads()):
            t0 = time.perf_counter()
            r = oracle.sample(m.verts, m.tris, m.bbox, m.w, axes="xyz", brute=brute, nthreads=nt)
            out[f"{mode}_{nt}_threads_s"] = round(time.perf_counter() - t0, 4)
    out["samples"] = sum(r[a].n for a in range(3))
    return out


def copy_bandwidth(torch, mib: int = 1024, reps: int = 10):
    """Device-to-device copy of ``mib`` MiB (read + write counted): the HBM
    ceiling a plain copy kernel reaches on this GPU."""
    src = torch.ones((mib << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    with Timer(torch) as t:
        for _ in range(reps):
            dst.copy_(src)
    gbs = 2 * (mib << 20) * reps / (t.ms / 1e3) / 1e9
    del src, dst
    return {"bytes_per_copy": 2 * (mib << 20), "GBps": round(gbs, 1),
            "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


class Timer:
    """HIP events on the current stream around a region, after a synchronise."""

    def __init__(self, torch):
        self.torch = torch

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.a = self.torch.cuda.Event(enable_timing=True)
        self.b = self.torch.cuda.Event(enable_timing=True)
        self.a.record()
        return self

    def __exit__(self, *exc):
        self.b.record()
        self.torch.cuda.synchronize()
        self.ms = self.a.elapsed_time(self.b)


def measure_plain(ldni, torch, mesh, steps, warmup, workload):
    verts = torch.from_numpy(mesh.verts).cuda()
    tris = torch.from_numpy(mesh.tris).cuda()

    def step():
        r = ldni.ldni_sample(verts, tris, mesh.bbox, mesh.w, "xyz")
        n = [int(r.view(a).n_samples) for a in range(3)]
        ml = [int(r.view(a).max_layers) for a in range(3)]
        r.free()
        return n, ml

    for _ in range(max(1, warmup)):
        n_axis, max_layers = step()
    # the timed steps run without per-launch events; a second pass times
    # every step on its own (percentiles), a third records an event pair
    # around every kernel launch on the library's stream for the per-kernel
    # durations
    with Timer(torch) as t:
        for _ in range(steps):
            n_axis, max_layers = step()
    ms_step = t.ms / steps
    per_step = []
    for _ in range(steps):
        with Timer(torch) as ts:
            step()
        per_step.append(ts.ms)
    ldni.profile_enable(True)
    with Timer(torch) as tp:
        for _ in range(steps):
            step()
    ldni.profile_enable(False)
    kstats = ldni.profile_read()
    samples = sum(n_axis)
    b = fwd_bytes(mesh, samples)
    dom_name, (dom_launches, dom_ms) = max(kstats.items(), key=lambda kv: kv[1][1])
    launches_per_step = max(1, dom_launches // steps)
    avg_s = dom_ms / dom_launches / 1e3
    # the measurement's roofline: the step's algorithmic bytes (mesh read
    # once, offsets and (depth, normal) samples written once) over the
    # dominant kernel's time per step, against the HBM peak
    dom_step_s = avg_s * launches_per_step
    achieved = b / dom_step_s / 1e9
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": read_traffic(workload, dom_name),
                "avg_launch_us": round(avg_s * 1e6, 2), "launches_per_step": launches_per_step,
                "algorithmic_bytes_per_step": b,
                "path": {"achieved": round(b / (ms_step / 1e3) / 1e9, 2),
                         "frac": round(b / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}}
    # arithmetic of the sampling pass against the vector FP64 peak: per
    # candidate pixel the exact coverage test, per hit the barycentric depth
    cand = candidate_count(mesh)
    flops = FLOPS_PER_CANDIDATE * cand + FLOPS_PER_HIT * samples
    sample_s = kstats["sample"][1] / steps / 1e3 if "sample" in kstats else dom_step_s
    alu = {"bound": "alu", "kernel": "sample", "unit": "TFLOP/s", "peak": FP64_PEAK_TFLOPS,
           "achieved": round(flops / sample_s / 1e12, 3),
           "frac": round(flops / sample_s / 1e12 / FP64_PEAK_TFLOPS, 4),
           "algorithmic_flops_per_step": flops, "candidates_per_step": cand}
    q = np.percentile(per_step, [10, 50, 90])
    return {
        "value": samples / (ms_step / 1e3),
        "ms_per_step": ms_step,
        "step_ms_p10_p50_p90": [round(float(x), 4) for x in q],
        "samples_per_step": samples,
        "samples_per_axis": n_axis,
        "max_layers": max_layers,
        "roofline": roofline,
        "alu_roofline": alu,
        "path_roofline": {"algorithmic_bytes_per_step": b,
                          "achieved_GBps": round(b / (ms_step / 1e3) / 1e9, 2),
                          "frac_of_hbm_peak": round(b / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_ms_per_step": {k: round(v[1] / steps, 4) for k, v in kstats.items()},
        "profiled_ms_per_step": round(tp.ms / steps, 4),
    }


def measure_rgb8(ldni, torch, mesh, steps):
    """The approximate normal output (Sec. 3, 8 bits per component, one packed
    word per sample) against float normals through the same torch-output
    call (ldni_sample_begin/finish)."""
    verts = torch.from_numpy(mesh.verts).cuda()
    tris = torch.from_numpy(mesh.tris).cuda()
    out = {}
    for kind in ("f32", "rgb8"):
        for _ in range(2):
            ldni.sample(verts, tris, mesh.bbox, mesh.w, "xyz", normals=kind)
        ldni.profile_enable(True)
        with Timer(torch) as t:
            for _ in range(steps):
                ldni.sample(verts, tris, mesh.bbox, mesh.w, "xyz", normals=kind)
        ldni.profile_enable(False)
        ks = ldni.profile_read()
        out[kind] = {"ms_per_step": round(t.ms / steps, 4),
                     "place_ms": round(ks["place"][1] / steps, 4) if "place" in ks else None}
    return {"bytes_per_sample": {"f32": 20, "rgb8": 12}, **out}


def measure_batch(ldni, torch, mg, reps):
    """256 seeded meshes, each at its own w: one graph replay vs 256 plain
    ldni_sample calls on one stream."""
    meshes = mg.c4_batch256()
    dev = [(torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.tris).cuda(), m) for m in meshes]
    b = ldni.sample_batch([(v, f, m.bbox, m.w) for v, f, m in dev], "xyz")
    samples = sum(int(b.view(k, a).n_samples) for k in range(len(dev)) for a in range(3))
    b.run()
    with Timer(torch) as t:
        for _ in range(reps):
            b.run()
    ms_batch = t.ms / reps

    def plain_all():
        n = 0
        for v, f, m in dev:
            r = ldni.ldni_sample(v, f, m.bbox, m.w, "xyz")
            n += sum(int(r.view(a).n_samples) for a in range(3))
            r.free()
        return n

    n_plain = plain_all()
    with Timer(torch) as t:
        for _ in range(reps):
            n_plain = plain_all()
    ms_plain = t.ms / reps
    b.free()
    return {
        "workload": "batch256",
        "description": "256 seeded flower/torus/icosphere meshes, triangle counts log-uniform "
                       "1e3..5e5, each at its own w in {64..1024}, 3 axes",
        "n_tris": int(sum(m.n_tris for m in meshes)),
        "sum_w2": int(sum(m.w * m.w for m in meshes)),
        "samples_per_step": samples,
        "batched": {"value": samples / (ms_batch / 1e3), "ms_per_step": round(ms_batch, 4)},
        "plain_256_calls": {"value": n_plain / (ms_plain / 1e3), "ms_per_step": round(ms_plain, 4)},
        "speedup": round(ms_plain / ms_batch, 3),
        "identical_sample_count": n_plain == samples,
    }


def measure_fwd_bwd(ldni, torch, mg, reps):
    """Flower at w=512: forward (torch-allocated outputs) and the backward of
    the squared-error loss to a perturbed copy's LDNI."""
    import numpy as np
    m = mg.c2_flower()
    tgt = mg.c5_target(m)
    v = torch.from_numpy(m.verts).cuda()
    f = torch.from_numpy(m.tris).cuda()
    tv = torch.from_numpy(tgt.verts).cuda()
    T = ldni.sample(tv, f, m.bbox, m.w, "xyz")
    R = ldni.sample(v, f, m.bbox, m.w, "xyz")
    gd, gn = {}, {}
    for a in range(3):
        c = R[a].counts().cpu().numpy()
        ct = T[a].counts().cpu().numpy()
        ro = R[a].offsets64().cpu().numpy()
        to = T[a].offsets64().cpu().numpy()
        pix = np.nonzero((c == ct) & (c > 0))[0]
        cnt = c[pix]
        k = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        s = torch.from_numpy(np.repeat(ro[pix], cnt) + k).cuda()
        st = torch.from_numpy(np.repeat(to[pix], cnt) + k).cuda()
        gd[a] = torch.zeros(R[a].n, device="cuda")
        gn[a] = torch.zeros(R[a].n, 3, device="cuda")
        gd[a][s] = 2 * (R[a].depth[s] - T[a].depth[st])
        gn[a][s] = 2 * (R[a].normal[s] - T[a].normal[st])
    samples = sum(R[a].n for a in range(3))
    g = torch.zeros_like(v)
    for _ in range(2):
        ldni.sample(v, f, m.bbox, m.w, "xyz")
        ldni.ldni_backward(v, f, m.bbox, m.w, R, gd, gn, grad_verts=g)
    with Timer(torch) as t:
        for _ in range(reps):
            ldni.sample(v, f, m.bbox, m.w, "xyz")
    ms_f = t.ms / reps
    ldni.profile_enable(True)
    with Timer(torch) as t:
        for _ in range(reps):
            ldni.ldni_backward(v, f, m.bbox, m.w, R, gd, gn, grad_verts=g)
    ldni.profile_enable(False)
    ms_b = t.ms / reps
    kb = ldni.profile_read().get("backward", (1, 0.0))
    bwd_bytes = 24 * m.n_verts + 12 * m.n_tris + 3 * 4 * (m.w * m.w + 1) + 20 * samples + 12 * m.n_verts
    return {
        "workload": "flower-512 forward+backward",
        "samples": samples,
        "forward_ms": round(ms_f, 4),
        "backward_ms": round(ms_b, 4),
        "bwd_over_fwd": round(ms_b / ms_f, 3),
        "value": samples / ((ms_f + ms_b) / 1e3),
        "backward_roofline": {"bound": "hbm", "algorithmic_bytes": bwd_bytes,
                              "achieved_GBps": round(bwd_bytes / (kb[1] / kb[0] / 1e3) / 1e9, 2)
                              if kb[1] > 0 else None,
                              "peak": HBM_PEAK_GBS,
                              "frac": round(bwd_bytes / (kb[1] / kb[0] / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
                              if kb[1] > 0 else None,
                              # counter bytes of one call (both backward kernels)
                              "traffic": read_traffic("flower-512-fwdbwd", "backward", "ldni_backward.hip")},
    }


def measure_boolean(ldni, torch, mg, reps):
    """Boolean operations (Sec. 4.1, small interval removal Sec. 4.1.1) of two
    seeded scenes sampled on one grid (scene64 seeds 1 and 7, w = 2048): one
    step is the union, intersection and difference on all three axes through
    the C ABI (nine calls, results freed)."""
    meshes = [mg.c3_scene64(seed=1), mg.c3_scene64(seed=7)]
    L = []
    for m in meshes:
        v = torch.from_numpy(m.verts).cuda()
        f = torch.from_numpy(m.tris).cuda()
        L.append(ldni.sample(v, f, m.bbox, m.w, "xyz"))
    del meshes
    w = L[0][0].w
    npix = w * w
    ops = ("union", "intersection", "difference")
    n_out, n_in = 0, 0
    for op in ops:
        for a in range(3):
            r = ldni.ldni_boolean(L[0][a], L[1][a], op)
            n_out += int(r.view(a).n_samples)
            n_in += L[0][a].n + L[1][a].n
            r.free()

    def step():
        for op in ops:
            for a in range(3):
                ldni.ldni_boolean(L[0][a], L[1][a], op).free()

    for _ in range(2):
        step()
    with Timer(torch) as t:
        for _ in range(reps):
            step()
    ms = t.ms / reps
    ldni.profile_enable(True)
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    ldni.profile_enable(False)
    ks = ldni.profile_read()
    calls = 9
    # algorithmic bytes: both inputs' offsets and depths, the kept samples'
    # normal and id, the result's offsets and samples
    alg = calls * 12 * (npix + 1) + 4 * n_in + 36 * n_out
    kern = {k: round(v[1] / reps, 4) for k, v in ks.items() if k.startswith("boolean")}
    # the count pass alone must read both inputs' offsets and depths and
    # write the counts; the write pass also the kept samples and the result
    cnt_bytes = calls * 12 * (npix + 1) + 4 * n_in
    wr_bytes = calls * 16 * (npix + 1) + 4 * n_in + 36 * n_out
    def roof(name, b):
        if name not in ks or ks[name][1] <= 0:
            return None
        gbs = b / (ks[name][1] / reps / 1e3) / 1e9
        # counter bytes per launch (the nine calls of a step average out
        # over whole steps) times the launches of a step
        per_launch = read_traffic("boolean-2048", name, "ldni_boolean.hip")
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_step": b,
                "traffic_per_step": calls * per_launch if per_launch is not None else None}
    return {
        "workload": "boolean-2048",
        "description": "union, intersection and difference of scene64 (seed 1) and scene64 (seed 7) "
                       "LDNIs at w=2048, 3 axes each",
        "input_samples_per_step": n_in, "output_samples_per_step": n_out,
        "ms_per_step": round(ms, 4),
        "value": n_in / (ms / 1e3), "unit": "input samples/s",
        "path_roofline": {"algorithmic_bytes_per_step": alg,
                          "achieved_GBps": round(alg / (ms / 1e3) / 1e9, 1),
                          "frac_of_hbm_peak": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "count_roofline": roof("boolean_count", cnt_bytes),
        "write_roofline": roof("boolean_write", wr_bytes),
        "kernels_ms_per_step": kern,
    }


def measure_nodes(ldni, torch, mg, reps):
    """Grid-node classification (Definition 3; Sec. 5.1 step 1) of the scene64
    LDNIs at w = 2048: one step is one ldni_classify_nodes call over all
    2048^3 nodes (the bit volume, 1 GiB, written in full)."""
    m = mg.c3_scene64(seed=1)
    v = torch.from_numpy(m.verts).cuda()
    f = torch.from_numpy(m.tris).cuda()
    L = ldni.sample(v, f, m.bbox, m.w, "xyz")
    del v, f
    w = m.w
    bits = torch.empty(ldni.node_words(w), dtype=torch.int32, device="cuda")
    _, n_in, n_split = ldni.classify_nodes([L[0], L[1], L[2]], m.bbox, bits)
    for _ in range(2):
        ldni.classify_nodes([L[0], L[1], L[2]], m.bbox, bits)
    with Timer(torch) as t:
        for _ in range(reps):
            ldni.classify_nodes([L[0], L[1], L[2]], m.bbox, bits)
    ms = t.ms / reps
    ldni.profile_enable(True)
    for _ in range(reps):
        ldni.classify_nodes([L[0], L[1], L[2]], m.bbox, bits)
    torch.cuda.synchronize()
    ldni.profile_enable(False)
    ks = ldni.profile_read()
    # algorithmic bytes: each LDNI's offsets and depths read once, the bit
    # volume written once
    n_samples = sum(L[a].n for a in range(3))
    alg = 3 * 4 * (w * w + 1) + 4 * n_samples + 4 * bits.numel()
    # the vote kernel's own algorithmic share: the bit volume it writes (the
    # span codes it reads are implementation traffic of the two-pass design)
    vote_alg = 4 * bits.numel()
    roof = None
    if "classify_nodes" in ks and ks["classify_nodes"][1] > 0:
        k_ms = ks["classify_nodes"][1] / reps
        gbs = vote_alg / (k_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": "classify_nodes", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                "traffic": read_traffic("nodes-2048", "classify_nodes", "ldni_nodes.hip"),
                "avg_launch_us": round(k_ms * 1e3, 2), "algorithmic_bytes_per_launch": vote_alg}
    kern = {k: round(v[1] / reps, 4) for k, v in ks.items() if k in ("node_codes", "classify_nodes")}
    return {
        "workload": "nodes-2048",
        "description": "inside/outside of the 2048^3 grid nodes of the scene64 (seed 1) LDNIs by the "
                       "two-of-three vote",
        "nodes_per_step": w ** 3, "input_samples": n_samples, "nodes_inside": n_in,
        "nodes_with_split_votes": n_split,
        "ms_per_step": round(ms, 4), "value": w ** 3 / (ms / 1e3), "unit": "nodes/s",
        "roofline": roof,
        "path_roofline": {"algorithmic_bytes_per_step": alg,
                          "achieved_GBps": round(alg / (ms / 1e3) / 1e9, 1),
                          "frac_of_hbm_peak": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_ms_per_step": kern,
    }


def measure_offset(ldni, torch, mg, reps):
    """Offsetting (Sec. 4.2) of the flower (the C2 mesh) sampled at w = 128
    (the paper's offsetting resolution) and w = 256: one step is an outer and
    an inner offset by two pixels (r = +2h, -2h), each a full ldni_offset
    call on resident LDNIs, results freed."""
    m = mg.c2_flower()
    v = torch.from_numpy(m.verts).cuda()
    f = torch.from_numpy(m.tris).cuda()
    out = {}
    for w in (128, 256):
        L = ldni.sample(v, f, m.bbox, w, "xyz")
        h = (m.bbox[3] - m.bbox[0]) / w
        n_in = sum(L[a].n for a in range(3))
        n_out = 0
        for r in (2 * h, -2 * h):
            res = ldni.ldni_offset(L, m.bbox, r)
            n_out += sum(int(res.view(a).n_samples) for a in range(3))
            res.free()

        def step():
            for r in (2 * h, -2 * h):
                ldni.ldni_offset(L, m.bbox, r).free()

        step()
        with Timer(torch) as t:
            for _ in range(reps):
                step()
        ms = t.ms / reps
        ldni.profile_enable(True)
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        ldni.profile_enable(False)
        ks = ldni.profile_read()
        kern = {k: round(val[1] / reps, 4) for k, val in ks.items() if k.startswith("offset")}
        # algorithmic bytes: the three LDNIs read (offsets, depth, normal, id), the results written
        alg = 2 * (3 * 4 * (w * w + 1) + 20 * n_in) + 3 * 4 * 2 * (w * w + 1) + 20 * n_out
        out[f"flower-{w}"] = {
            "w": w, "r_pixels": 2, "input_samples": n_in, "output_samples_per_step": n_out,
            "ms_per_step": round(ms, 4), "ms_per_offset": round(ms / 2, 4),
            "value": 2 * n_in / (ms / 1e3), "unit": "input samples offset/s",
            "path_roofline": {"algorithmic_bytes_per_step": alg,
                              "achieved_GBps": round(alg / (ms / 1e3) / 1e9, 1),
                              "frac_of_hbm_peak": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 5)},
            "kernels_ms_per_step": kern,
        }
        del L
    out["description"] = ("outer and inner offset (r = +2h, -2h) of the flower mesh's LDNIs: union with "
                          "(difference of) a sphere at every sample, all three axes")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=None,
                    choices=sorted(PLAIN) + ["batch256", "flower-512-fwdbwd", "boolean-2048", "nodes-2048",
                                                "offset-flower"],
                    help="measure one part only (default: the headline plus every part)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile", default=None, help="tile shape TWxTH")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before warm-up, copy a buffer of this many MiB once (a plain copy "
                         "kernel of known size, to scale hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} refused: LDNI sampling here runs on one GPU; "
              "the multi-GPU split (by axis or by pixel-row band) is a design note only.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1009_0794_amd as ldni
    from paper_1009_0794_amd import meshgen as mg

    torch.cuda.set_device(0)
    if args.tile:
        tw, th = (int(x) for x in args.tile.lower().split("x"))
        ldni.set_tile_shape(tw, th)
    if args.calib_copy_mib > 0:
        src = torch.ones((args.calib_copy_mib << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    head = args.workload if args.workload in PLAIN else "scene64-2048"
    line = {"metric": METRIC, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 out, f64 internal",
            "data": "synthetic (seeded meshes from paper_1009_0794_amd/meshgen.py)"}
    if args.workload in (None, *PLAIN):
        mesh = getattr(mg, PLAIN[head][0])()
        r = measure_plain(ldni, torch, mesh, args.steps, args.warmup, head)
        line.update({"value": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                     "config": {"workload": head, "description": PLAIN[head][1], "n_tris": mesh.n_tris,
                                "n_verts": mesh.n_verts, "w": mesh.w, "axes": "xyz",
                                "samples_per_step": r["samples_per_step"],
                                "samples_per_axis": r["samples_per_axis"], "max_layers": r["max_layers"],
                                "parallelism": "single GPU"},
                     "step_ms_p10_p50_p90": r["step_ms_p10_p50_p90"],
                     "roofline": r["roofline"], "alu_roofline": r["alu_roofline"],
                     "path_roofline": r["path_roofline"],
                     "kernels_ms_per_step": r["kernels_ms_per_step"]})
        line["hbm_copy_probe"] = copy_bandwidth(torch)
        probe = atomic_probe(torch)
        req = read_atomics(head)
        ks = r["kernels_ms_per_step"]
        line["atomics"] = {"probe": probe, "kernels": {
            k: {"requests_per_launch": int(n), "G_per_s": round(n / (ks[k] / 1e3) / 1e9, 3) if ks.get(k) else None,
                "frac_of_probe": round(n / (ks[k] / 1e3) / 1e9 / probe["G_per_s"], 4) if ks.get(k) else None}
            for k, n in req.items()}}
        line["normal_rgb8"] = measure_rgb8(ldni, torch, mesh, max(2, args.steps // 2))
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline(mesh, args.cpu_seconds)
        del mesh
    if args.workload is None:
        c1 = mg.c1_icosphere()
        r1 = measure_plain(ldni, torch, c1, args.steps, args.warmup, "icosphere-128")
        line["icosphere_128"] = {"value": round(r1["value"], 1), "ms_per_step": round(r1["ms_per_step"], 4),
                                 "step_ms_p10_p50_p90": r1["step_ms_p10_p50_p90"],
                                 "samples_per_step": r1["samples_per_step"],
                                 "path_roofline": r1["path_roofline"],
                                 "kernels_ms_per_step": r1["kernels_ms_per_step"]}
        if not args.no_cpu_baseline:
            line["icosphere_128"]["oracle_seconds"] = oracle_c1_seconds()
        fl = mg.c2_flower()
        r2 = measure_plain(ldni, torch, fl, args.steps, args.warmup, "flower-512")
        line["flower_512"] = {"value": round(r2["value"], 1), "ms_per_step": round(r2["ms_per_step"], 4),
                              "step_ms_p10_p50_p90": r2["step_ms_p10_p50_p90"],
                              "samples_per_step": r2["samples_per_step"],
                              "path_roofline": r2["path_roofline"], "roofline": r2["roofline"],
                              "kernels_ms_per_step": r2["kernels_ms_per_step"]}
    if args.workload in (None, "batch256"):
        rb = measure_batch(ldni, torch, mg, reps=max(1, args.steps // 4))
        if args.workload == "batch256":
            line.update({"value": round(rb["batched"]["value"], 1),
                         "ms_per_step": rb["batched"]["ms_per_step"],
                         "config": {"workload": "batch256", "description": rb["description"],
                                    "parallelism": "single GPU"}})
        line["batched"] = rb
    if args.workload in (None, "flower-512-fwdbwd"):
        rf = measure_fwd_bwd(ldni, torch, mg, reps=args.steps)
        if args.workload == "flower-512-fwdbwd":
            line.update({"value": round(rf["value"], 1),
                         "ms_per_step": round(rf["forward_ms"] + rf["backward_ms"], 4),
                         "config": {"workload": "flower-512 forward+backward",
                                    "parallelism": "single GPU"}})
        line["fwd_bwd"] = rf
    if args.workload in (None, "boolean-2048"):
        ro = measure_boolean(ldni, torch, mg, reps=max(2, args.steps // 4))
        if args.workload == "boolean-2048":
            line.update({"value": round(ro["value"], 1), "ms_per_step": ro["ms_per_step"],
                         "config": {"workload": "boolean-2048", "description": ro["description"],
                                    "parallelism": "single GPU"}})
        line["boolean"] = ro
    if args.workload in (None, "nodes-2048"):
        rn = measure_nodes(ldni, torch, mg, reps=max(2, args.steps // 4))
        if args.workload == "nodes-2048":
            line.update({"value": round(rn["value"], 1), "unit": rn["unit"], "ms_per_step": rn["ms_per_step"],
                         "config": {"workload": "nodes-2048", "description": rn["description"],
                                    "parallelism": "single GPU"}})
        line["nodes"] = rn
    if args.workload in (None, "offset-flower"):
        rf2 = measure_offset(ldni, torch, mg, reps=max(2, args.steps // 4))
        if args.workload == "offset-flower":
            line.update({"value": round(rf2["flower-256"]["value"], 1), "unit": rf2["flower-256"]["unit"],
                         "ms_per_step": rf2["flower-256"]["ms_per_step"],
                         "config": {"workload": "offset-flower-256", "description": rf2["description"],
                                    "parallelism": "single GPU"}})
        line["offset"] = rf2
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
