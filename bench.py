"""Benchmark: CWENO reconstruction throughput on one MI355X.

Workload: 2-D, degree M = 3 (10 basis functions), 512 x 512 x 2 = 524,288
jittered periodic triangles, central stencil n_e = 20, 3 sectors, 9 ideal-MHD-
shaped variables (smooth 8-mode Fourier fields plus a planar jump with density
ratio 10).  One step = one cweno_reconstruct of the whole mesh (all five steps
of the method for every cell and variable), inputs already resident in HBM.

Prints one JSON line.  ``value`` is the FP64 path's cells*vars/s; the FP32
operator path is reported beside it under "fp32".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CWENO cells·vars reconstructed/s + % HBM peak, FP64 vs FP32; p99 latency"
HBM_PEAK_GBS = 8000.0
SEED = 16120935
KERNEL_SRC = os.path.join(ROOT, "paper_1612_09335_amd", "csrc", "reconstruct_kernel.hpp")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_cell(d, M, n_e, G, nv, s_op, s_io):
    """Bytes one reconstruction must move per cell with precomputed operators.

    operators s_op*[(nb-1)(n_e-1) + (d+1)d^2], int32 gather list 4*G, uint8
    sector positions (d+1)d and sector mask 1, averages read once nv*s_io,
    coefficients written once nv*nb*s_io.
    """
    nb = (M + 1) * (M + 2) // 2 if d == 2 else (M + 1) * (M + 2) * (M + 3) // 6
    return (s_op * ((nb - 1) * (n_e - 1) + (d + 1) * d * d) + 4 * G + (d + 1) * d + 1
            + nv * s_io + nv * nb * s_io)


def kernel_source_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def load_traffic(tag):
    """HBM bytes per launch measured by rocprofv3 counters, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(tag)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_source_sha") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def time_path(torch, mesh, q, steps, warmup):
    out = torch.empty((q.shape[0], mesh.n_basis, mesh.n_cells), dtype=q.dtype, device=q.device)
    mesh.tune(q, out, repeats=5)            # the library's autotuner picks the kernel variant
    for _ in range(warmup):
        mesh.reconstruct(q, out=out)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record()
        mesh.reconstruct(q, out=out)
        ends[k].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])     # ms
    total = starts[0].elapsed_time(ends[-1])                               # ms
    return dict(total_ms=total, per_ms=per, wall_s=wall, out=out)


def cpu_baseline(m, Q, degree, factor, budget_s):
    """The CPU oracle on a bounded sample of the same workload's cells."""
    from threadpoolctl import threadpool_limits

    from oracle import CwenoOracle, Options
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=degree, stencil_factor=factor))
    rng = np.random.default_rng(SEED)
    cells = rng.permutation(m.n_cells)
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s and done < len(cells):
            o.reconstruct_cell(int(cells[done]), Q)
            done += 1
        dt = time.perf_counter() - t0
    return dict(value=done * Q.shape[0] / dt, unit="cells·vars/s", cores=1, kind="oracle",
                sample=f"{done} random cells of the benchmark mesh (all {Q.shape[0]} variables), "
                       f"one thread, {dt:.1f} s; oracle set-up (face adjacency) excluded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": a.numel() * 8, "launches": 3}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the reconstruction of a mesh runs on a single device "
              "(multi-GPU sharding is a design note, not implemented); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_09335_amd as C
    from synthetic import tri_mesh, workload_fields

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    d, M, n, factor = 2, 3, 512, 0.0
    log("generating mesh and fields")
    m = tri_mesh(n, 0.15, SEED)
    Q = workload_fields(m, "mhd2d", SEED)
    nv = Q.shape[0]
    log("precompute")
    t0 = time.perf_counter()
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, stencil_factor=factor, ops="both")
    t_pre = time.perf_counter() - t0
    log(f"precompute {t_pre:.2f} s, n_e={lm.n_e}, gather={lm.gather_len}, device bytes={lm.device_bytes}")
    q64 = torch.tensor(Q, dtype=torch.float64, device=dev)
    q32 = q64.float()

    res = {}
    for tag, q, s in (("f64", q64, 8), ("f32", q32, 4)):
        log(f"timing {tag}")
        r = time_path(torch, lm, q, args.steps, args.warmup)
        got = r["out"][:, 0].cpu().numpy()
        assert np.array_equal(got, q.cpu().numpy()), "coefficient 0 must copy the input"
        bpc = algorithmic_bytes_per_cell(d, M, lm.n_e, lm.gather_len, nv, s, s)
        bytes_launch = bpc * m.n_cells
        ms = r["total_ms"] / args.steps
        kern_ms = float(np.mean(r["per_ms"]))
        achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
        traffic = load_traffic(tag)
        res[tag] = dict(
            value=m.n_cells * nv / (ms * 1e-3), ms_per_step=ms,
            latency_ms=dict(p50=float(np.percentile(r["per_ms"], 50)), p99=float(np.percentile(r["per_ms"], 99))),
            roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                          algorithmic_bytes_per_cell=bpc, algorithmic_bytes_per_launch=bytes_launch))
        res[tag]["variant"] = lm.get_variant(tag, nv)
        log(f"{tag}: variant {res[tag]['variant']}, {ms:.4f} ms/step, {res[tag]['value']:.3e} cells*vars/s, {achieved:.0f} GB/s "
            f"({100 * achieved / HBM_PEAK_GBS:.1f}% of peak)")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(m, Q, M, factor, args.cpu_seconds)
        log(f"cpu: {cpu['value']:.3e} cells*vars/s")

    r64 = res["f64"]
    line = {
        "metric": METRIC, "value": r64["value"], "unit": "cells·vars/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "CWENO 2-D M=3 (10 basis functions), 524,288 jittered periodic triangles "
                               "(512x512x2), n_e=20, 3 sectors, 9 MHD-shaped variables",
                   "cells": m.n_cells, "n_vars": nv, "degree": M, "dim": d, "n_e": lm.n_e,
                   "lambda0": 0.95, "eps": 1e-14, "r": 4, "seed": SEED},
        "roofline": r64["roofline"],
        "latency_ms": r64["latency_ms"],
        "kernel_variant": {"f64": res["f64"]["variant"], "f32": res["f32"]["variant"]},
        "fp32": {"value": res["f32"]["value"], "ms_per_step": res["f32"]["ms_per_step"],
                 "latency_ms": res["f32"]["latency_ms"], "roofline": res["f32"]["roofline"],
                 "dtype": "f32"},
        "cpu_baseline": cpu,
        "precompute_s": t_pre,
        "kernel_source_sha": kernel_source_hash(),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
