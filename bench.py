#!/usr/bin/env python3
"""Throughput of LDNI sampling on one MI355X.

One step = one pass of the sampling path (triangle setup, tile binning, count,
scan, write + per-pixel sort, for all three axes) over the workload's mesh,
through the C ABI call ``ldni_sample`` (library-owned outputs from the
stream-ordered pool) followed by ``ldni_free``.  Inputs are resident in HBM
before the timed region starts.  The metric is LDNI samples written per
second, summed over the three axes.

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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

WORKLOADS = {
    # name: (mesh builder, description)
    "scene64-2048": ("c3_scene64", "64 disjoint closed shells, 2,152,448 triangles, up to 32 layers, w=2048, 3 axes"),
    "flower-512": ("c2_flower", "seeded flower UV sphere 512x256, 261,120 triangles, w=512, 3 axes"),
    "icosphere-128": ("c1_icosphere", "icosphere level 3, 1,280 triangles, w=128, 3 axes"),
}


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_1009_0794_amd", "csrc", "ldni_kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def read_traffic(workload: str, kernel: str, launches_per_step: int):
    """HBM bytes per launch of ``kernel`` from the committed counter summary,
    or None if there is none or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_kernel_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def algorithmic_bytes(mesh, n_axes):
    """What the method must move (read the mesh once, write offsets and
    (depth, normal) samples once), per kernel that moves it."""
    V, T, w = mesh.n_verts, mesh.n_tris, mesh.w
    return {
        "setup": 12 * V + 12 * T,
        "scan_pixels": 4 * (w * w + 1) * n_axes,
        "write": None,  # 16 bytes per sample, filled in once the counts are known
    }


def cpu_baseline(mesh, seconds: float):
    """The oracle on the same workload, all three axes, repeated until about
    ``seconds`` of CPU work; its mean rate."""
    import oracle
    threads = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        threads = min(threads, int(env))
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
    return {
        "value": samples / elapsed,
        "unit": "samples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"the whole workload (3 axes, culled mode) {passes} time(s): "
                  f"{samples} samples in {elapsed:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="scene64-2048", choices=sorted(WORKLOADS))
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

    builder, desc = WORKLOADS[args.workload]
    mesh = getattr(mg, builder)()
    if args.tile:
        tw, th = (int(x) for x in args.tile.lower().split("x"))
        ldni.set_tile_shape(tw, th)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    verts = torch.from_numpy(mesh.verts).to(dev)
    tris = torch.from_numpy(mesh.tris).to(dev)
    torch.cuda.synchronize()

    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        r = ldni.ldni_sample(verts, tris, mesh.bbox, mesh.w, "xyz")
        n = [int(r.view(a).n_samples) for a in range(3)]
        ml = [int(r.view(a).max_layers) for a in range(3)]
        r.free()
        return n, ml

    for _ in range(args.warmup):
        n_axis, max_layers = step()
    if args.warmup == 0:
        n_axis, max_layers = step()
    torch.cuda.synchronize()

    ldni.profile_enable(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record()
    total = 0
    for _ in range(args.steps):
        n_axis, max_layers = step()
        total += sum(n_axis)
    stop.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ldni.profile_enable(False)
    kstats = ldni.profile_read()
    ms = start.elapsed_time(stop)
    ms_per_step = ms / args.steps
    samples_per_step = sum(n_axis)
    value = total / (ms / 1e3)

    # roofline of the dominant kernel
    alg = algorithmic_bytes(mesh, 3)
    alg["write"] = 16 * samples_per_step
    dom = max(kstats.items(), key=lambda kv: kv[1][1])
    dom_name, (dom_launches, dom_ms) = dom
    per_step_launches = max(1, dom_launches // args.steps)
    avg_launch_s = dom_ms / dom_launches / 1e3
    alg_per_launch = alg.get(dom_name)
    if alg_per_launch is not None:
        alg_per_launch = alg_per_launch / per_step_launches
    achieved = (alg_per_launch / avg_launch_s / 1e9) if alg_per_launch else 0.0
    traffic = read_traffic(args.workload, dom_name, per_step_launches)
    roofline = {
        "bound": "hbm",
        "kernel": dom_name,
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "avg_launch_us": round(avg_launch_s * 1e6, 2),
        "algorithmic_bytes_per_launch": alg_per_launch,
    }
    b_fwd = 12 * mesh.n_verts + 12 * mesh.n_tris + 3 * 4 * (mesh.w * mesh.w + 1) + 16 * samples_per_step
    path = {
        "algorithmic_bytes_per_step": b_fwd,
        "achieved_GBps": round(b_fwd / (ms_per_step / 1e3) / 1e9, 2),
        "frac_of_hbm_peak": round(b_fwd / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
    }

    line = {
        "metric": "LDNI samples written/sec (3 axes) at w=512/2048; batched vs plain; fwd+bwd",
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 out, f64 internal",
        "data": "synthetic (seeded meshes generated in paper_1009_0794_amd/meshgen.py)",
        "config": {
            "workload": args.workload,
            "description": desc,
            "n_tris": mesh.n_tris,
            "n_verts": mesh.n_verts,
            "w": mesh.w,
            "axes": "xyz",
            "samples_per_step": samples_per_step,
            "samples_per_axis": n_axis,
            "max_layers": max_layers,
            "parallelism": "single GPU",
        },
        "roofline": roofline,
        "path_roofline": path,
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in kstats.items()},
        "wall_s": round(t_wall, 3),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(mesh, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
