"""Benchmark: CWENO reconstruction throughput on one MI355X.

Workload: 2-D, degree M = 3 (10 basis functions), 512 x 512 x 2 = 524,288
jittered periodic triangles, central stencil n_e = 20, 3 sectors, 9 ideal-MHD-
shaped variables (smooth 8-mode Fourier fields plus a planar jump with density
ratio 10).  One step = one cweno_reconstruct of the whole mesh (all five steps
of the method for every cell and variable), inputs already resident in HBM.

Prints one JSON line.  ``value`` is the FP64 path's cells*vars/s; the FP32
operator path is reported beside it under "fp32".  Unless --quick is given,
more workloads are measured and reported under "extras": the small 2-D M=2
mesh (8,192 triangles, 4 Euler variables) as launch latency p50/p99, the 3-D
M=3 mesh (1,572,864 Kuhn tetrahedra, 5 variables) as throughput, and (unless
--no-batch) a batch of 64 uneven meshes of mixed dimension and degree as one
FP32 graph launch against per-mesh FP64 launches, (unless
--serve-seconds 0) the serving loop: 200 registered meshes, an HBM budget
that holds their FP32 operators but not their FP64 ones, Poisson request
arrivals; latency p50/p99/p99.9 against a serial FP64 server, and (unless --no-moving) the moving-mesh path on the 2-D
and 3-D workloads with moved vertices: operators rebuilt from the vertices
in every call, FP64 arithmetic, against the stored-operator path.  The point
values of the benchmark reconstruction at the face Gauss points are timed
with every run, and (unless --no-weno) the classical unstructured WENO scheme
the paper compares CWENO with runs on the benchmark workload (memory and time
against CWENO).
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
FP64_VECTOR_TFS = 78.6
SEED = 16120935
CSRC = os.path.join(ROOT, "paper_1612_09335_amd", "csrc")
KERNEL_SRCS = ["reconstruct_kernel.hpp", "halo_kernel.hpp", "dispatch.hpp", "kernels.hip", "gen_sigma.cpp"]
MOVING_SRCS = ["moving_kernel.hpp", "moving.hpp", "moving_kernels.hip"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def n_basis(d, M):
    return (M + 1) * (M + 2) // 2 if d == 2 else (M + 1) * (M + 2) * (M + 3) // 6


def algorithmic_bytes_per_cell(d, M, n_e, nv, s):
    """Bytes one reconstruction must move per cell with precomputed operators.

    s [(nb-1)(n_e-1) + (d+1) d^2] operator entries, 4 (n_e-1) bytes of int32
    stencil indices, d (d+1) bytes of sector positions, and per variable the
    average read once and the nb coefficients written once.
    """
    nb = n_basis(d, M)
    return s * ((nb - 1) * (n_e - 1) + (d + 1) * d * d) + 4 * (n_e - 1) + d * (d + 1) + nv * s * (1 + nb)


def gm_points(d, M):
    """Points of the Grundmann-Moller rule exact to degree M on the d-simplex."""
    from math import comb
    s = M // 2
    return sum(comb(s - i + d, d) for i in range(s + 1))


def moving_flops_per_cell(d, M, n_e, nv):
    """FP64 operations one moving-mesh reconstruction spends per cell.

    Quadrature of the rows: (n_e-1) cells x nq points x (8 per basis function
    evaluated + 2 per accumulated average); Householder QR of the
    (n_e-1) x (nb-1) matrix, 2 m n^2 - 2/3 n^3; per variable the reflections
    (4 per entry of the lower trapezoid) and the back substitution (n^2), and
    the blend (the quadratic form, n^2, plus 10 per polynomial).
    """
    nb = n_basis(d, M)
    m, n = n_e - 1, nb - 1
    quad = m * gm_points(d, M) * (8 * nb + 2 * n)
    qr = 2 * m * n * n - 2 * n ** 3 / 3
    per_var = 4 * (m * n - n * (n - 1) / 2) + n * n + n * n + 10 * (d + 2)
    return quad + qr + nv * per_var


def measure_moving(torch, C, m, Q, M, label, d, steps, stored_ms):
    """Moving-mesh path: operators rebuilt from moved vertices in every call."""
    from synthetic import moved_vertices
    dev = torch.device("cuda:0")
    nv = Q.shape[0]
    t0 = time.perf_counter()
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops="none", moving=True)
    t_reg = time.perf_counter() - t0
    V = torch.tensor(moved_vertices(m, 0.2, 0.1), device=dev)
    flops = moving_flops_per_cell(d, M, lm.n_e, nv) * m.n_cells
    out = {"workload": f"{label} with every vertex moved (smooth periodic shear, gradient 0.2); stencils of the "
                       f"connectivity, operators rebuilt per call", "registration_s": t_reg,
           "device_bytes": lm.device_bytes, "flops_per_launch": flops}
    fault = torch.zeros(1, dtype=torch.int32, device=dev)
    for tag, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        q = torch.tensor(Q, dtype=tdt, device=dev)
        o = torch.empty((nv, lm.n_basis, lm.n_cells), dtype=tdt, device=dev)
        ms = time_loop(torch, lambda: lm.reconstruct_moving(V, q, out=o, fault=fault), steps, 2)
        tf = flops / (ms * 1e-3) / 1e12
        out[tag] = {"ms_per_step": ms, "value": m.n_cells * nv / (ms * 1e-3),
                    "vs_stored_operators": ms / stored_ms[tag],
                    "roofline": dict(bound="alu", achieved=tf, peak=FP64_VECTOR_TFS, unit="TFLOP/s",
                                     frac=tf / FP64_VECTOR_TFS,
                                     traffic=load_traffic("moving_" + tag, MOVING_SRCS) if d == 2 else None)}
        log(f"moving {label} {tag}: {ms:.3f} ms ({out[tag]['value']:.3e} cells*vars/s, {tf:.2f} TFLOP/s FP64, "
            f"{ms / stored_ms[tag]:.1f}x the stored-operator launch)")
        del q, o
    out["fault"] = int(fault.item())
    return out


def face_gauss_points(d, n):
    """n-point Gauss-Legendre points on every edge of the reference triangle (d = 2)."""
    g, _ = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (g + 1.0)
    verts = np.vstack([np.zeros(d), np.eye(d)])
    return np.vstack([np.outer(1 - t, verts[a]) + np.outer(t, verts[b])
                      for a in range(d + 1) for b in range(a + 1, d + 1)])


def measure_evaluate(torch, C, lm, Q, M, d, steps):
    """Point values of the benchmark reconstruction at the face Gauss points."""
    P = face_gauss_points(d, M + 1)
    pts = C.Points(d, M, P)
    nv, nb = Q.shape[0], lm.n_basis
    out = {"workload": f"coefficients of the benchmark reconstruction evaluated at {len(P)} face points "
                       f"({M + 1} Gauss-Legendre points on each edge)", "n_points": len(P)}
    for tag, tdt, s in (("f64", torch.float64, 8), ("f32", torch.float32, 4)):
        q = torch.tensor(Q, dtype=tdt, device="cuda:0")
        co = lm.reconstruct(q)
        vals = torch.empty((nv, len(P), lm.n_cells), dtype=tdt, device="cuda:0")
        ms = time_loop(torch, lambda: lm.evaluate(pts, co, out=vals), steps, 3)
        alg = lm.n_cells * nv * s * (nb + len(P))
        gbs = alg / (ms * 1e-3) / 1e9
        ms_two = time_loop(torch, lambda: (lm.reconstruct(q, out=co), lm.evaluate(pts, co, out=vals)), steps, 3)
        ms_fused = time_loop(torch, lambda: lm.reconstruct_points(pts, q, out=vals), steps, 3)
        fused_alg = (algorithmic_bytes_per_cell(d, M, lm.n_e, nv, s) + nv * s * (len(P) - nb)) * lm.n_cells
        out[tag] = {"ms_per_step": ms, "value": lm.n_cells * nv / (ms * 1e-3),
                    "roofline": dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                                     frac=gbs / HBM_PEAK_GBS, traffic=None, algorithmic_bytes_per_launch=alg),
                    "reconstruct_then_evaluate_ms": ms_two, "fused_ms": ms_fused,
                    "fused_roofline": dict(bound="hbm", achieved=fused_alg / (ms_fused * 1e-3) / 1e9,
                                           peak=HBM_PEAK_GBS, unit="GB/s",
                                           frac=fused_alg / (ms_fused * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                           algorithmic_bytes_per_launch=fused_alg)}
        log(f"evaluate {tag}: {ms:.4f} ms, {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM peak); "
            f"reconstruct + evaluate {ms_two:.4f} ms, fused {ms_fused:.4f} ms "
            f"({100 * out[tag]['fused_roofline']['frac']:.1f}% of HBM peak)")
        del q, co, vals
    return out


def measure_weno(torch, C, m, Q, M, d, steps, cweno_ms, cweno_n_e):
    """The classical unstructured WENO scheme on the benchmark workload (FP64)."""
    nv = Q.shape[0]
    t0 = time.perf_counter()
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, weno=True)
    t_pre = time.perf_counter() - t0
    nb, n_e, n_s = lm.n_basis, lm.n_e, 1 + 2 * (d + 1)
    nl, ne1 = nb - 1, n_e - 1
    vbmax = 4 if nl <= 9 else (2 if nl <= 19 else 1)
    passes = -(-nv // (8 * vbmax))        # up to 8 lanes per cell, vbmax variables each, per pass
    weno_entries = n_s * nl * ne1
    cweno_entries = nl * (cweno_n_e - 1) + (d + 1) * d * d
    alg = (8 * weno_entries + 4 * n_s * ne1 + 2 + nv * 8 * (1 + nb)) * m.n_cells
    streamed = (passes * (8 * weno_entries + 4 * n_s * ne1 + 2) + nv * 8 * (1 + nb)) * m.n_cells
    q = torch.tensor(Q, device="cuda:0")
    out = torch.empty((nv, nb, lm.n_cells), dtype=torch.float64, device="cuda:0")
    ms = time_loop(torch, lambda: lm.reconstruct(q, out=out), steps, 3)
    gbs = alg / (ms * 1e-3) / 1e9
    M_ = nb
    paper_ratio = ((1 + 2 * (d + 1)) * d * M_ * M_) / (d * M_ * M_ + (d + 1) * (d + 1) ** 2)
    r = {"workload": f"classical unstructured WENO on the benchmark mesh: {n_s} stencils of n_e={n_e} cells "
                     f"(central, {d + 1} forward and {d + 1} reverse cone sectors), degree {M} each, FP64",
         "precompute_s": t_pre, "device_bytes": lm.device_bytes, "n_dropped": lm.n_dropped,
         "operator_entries_per_cell": weno_entries, "cweno_operator_entries_per_cell": cweno_entries,
         "memory_ratio_weno_over_cweno": weno_entries / cweno_entries,
         "paper_formula_ratio": paper_ratio,
         "ms_per_step": ms, "value": m.n_cells * nv / (ms * 1e-3),
         "time_ratio_weno_over_cweno_f64": ms / cweno_ms, "operator_passes": passes,
         "roofline": dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                          traffic=None, algorithmic_bytes_per_launch=alg, streamed_bytes_per_launch=streamed,
                          streamed_frac=streamed / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)}
    log(f"weno: precompute {t_pre:.1f} s, {lm.device_bytes / 1e9:.2f} GB on the device, {ms:.3f} ms "
        f"({ms / cweno_ms:.1f}x CWENO FP64), operators {weno_entries / cweno_entries:.2f}x CWENO's "
        f"(paper formula {paper_ratio:.2f}x), streamed {100 * r['roofline']['streamed_frac']:.1f}% of HBM peak")
    del lm, q, out
    return r


def kernel_source_hash(names=KERNEL_SRCS):
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(tag, names=KERNEL_SRCS):
    """HBM bytes per launch measured by rocprofv3 counters, if still current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(tag)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_source_sha") != kernel_source_hash(names):
        return None
    return rec.get("bytes_per_launch")


def time_path(torch, mesh, q, steps, warmup, tune=True):
    out = torch.empty((q.shape[0], mesh.n_basis, mesh.n_cells), dtype=q.dtype, device=q.device)
    if tune:
        mesh.tune(q, out, repeats=5)        # the library's autotuner picks the kernel variant
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


def time_flushed(torch, mesh, q, out, steps, flush):
    """Per-launch ms with a 1 GiB overwrite between launches (the 256 MB
    Infinity Cache and the L2s hold none of the operators when a launch starts)."""
    times = []
    for _ in range(steps):
        flush.fill_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mesh.reconstruct(q, out=out)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def measure(torch, C, m, Q, M, factor, steps, warmup, label, d):
    """Time both precisions on one workload; returns per-precision records."""
    dev = torch.device("cuda:0")
    nv = Q.shape[0]
    t0 = time.perf_counter()
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, stencil_factor=factor, ops="both")
    t_pre = time.perf_counter() - t0
    log(f"{label}: precompute {t_pre:.2f} s, n_e={lm.n_e}, gather={lm.gather_len}, device bytes={lm.device_bytes}")
    res = {"precompute_s": t_pre, "n_e": lm.n_e, "mesh": lm}
    if lm.n_e <= 65:
        # the same operators assembled on the GPU from the host's stencils
        t0 = time.perf_counter()
        dm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, stencil_factor=factor, ops="both",
                    device_operators=True)
        torch.cuda.synchronize()
        res["precompute_device_operators_s"] = time.perf_counter() - t0
        log(f"{label}: registration with operators assembled on the GPU {res['precompute_device_operators_s']:.2f} s")
        del dm
    q64 = torch.tensor(Q, dtype=torch.float64, device=dev)
    for tag, q, s in (("f64", q64, 8), ("f32", q64.float(), 4)):
        r = time_path(torch, lm, q, steps, warmup)
        got = r["out"][:, 0].cpu().numpy()
        assert np.array_equal(got, q.cpu().numpy()), "coefficient 0 must copy the input"
        bpc = algorithmic_bytes_per_cell(d, M, lm.n_e, nv, s)
        bytes_launch = bpc * m.n_cells
        ms = r["total_ms"] / steps
        kern_ms = float(np.mean(r["per_ms"]))
        achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
        flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        ms_flushed = time_flushed(torch, lm, q, r["out"], max(10, steps // 5), flush)
        del flush
        res[tag] = dict(
            value=m.n_cells * nv / (ms * 1e-3), ms_per_step=ms, kernel_ms=kern_ms,
            flushed_ms=ms_flushed, flushed_frac=bytes_launch / (ms_flushed * 1e-3) / 1e9 / HBM_PEAK_GBS,
            latency_ms=dict(p50=float(np.percentile(r["per_ms"], 50)), p99=float(np.percentile(r["per_ms"], 99))),
            roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=achieved / HBM_PEAK_GBS, traffic=None,
                          algorithmic_bytes_per_cell=bpc, algorithmic_bytes_per_launch=bytes_launch),
            variant=lm.get_variant(tag, min(nv, 9)))
        log(f"{label} {tag}: variant {res[tag]['variant']}, {ms:.4f} ms/step, {res[tag]['value']:.3e} cells*vars/s, "
            f"{achieved:.0f} GB/s ({100 * achieved / HBM_PEAK_GBS:.1f}% of peak); cache-flushed launch "
            f"{ms_flushed:.4f} ms ({100 * res[tag]['flushed_frac']:.1f}%)")
    return res


def time_loop(torch, fn, steps, warmup):
    """Average ms of fn() over `steps` back-to-back calls on the current stream."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def measure_batch(torch, C, steps):
    """64 uneven meshes (seeded recipe): FP32 batch graph vs per-mesh launches."""
    from synthetic import batch_spec, workload_fields, workload_mesh
    spec = batch_spec()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    raw = [(workload_mesh(d, n, sd), M, sd) for d, n, M, sd in spec]
    Qs = [workload_fields(m, "smooth_jump", sd) for m, M, sd in raw]
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    meshes = [C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops="both") for m, M, sd in raw]
    t_pre = time.perf_counter() - t0
    cells = sum(m.n_cells for m, _, _ in raw)
    cv = sum(m.n_cells * Q.shape[0] for (m, _, _), Q in zip(raw, Qs))
    log(f"batch: {len(meshes)} meshes, {cells} cells, inputs {t_gen:.1f} s, precompute {t_pre:.1f} s")
    out = {"workload": f"{len(meshes)} jittered periodic meshes, cell counts log-uniform on [1e3, 3e5] "
                       f"({cells} cells), d in {{2,3}}, M in {{2,3,4}}, nv = d+2, smooth fields plus a jump",
           "cells": cells, "cells_vars": cv, "precompute_s": t_pre}
    for tag, tdt, s in (("f32", torch.float32, 4), ("f64", torch.float64, 8)):
        qs = [torch.tensor(Q, dtype=tdt, device=dev) for Q in Qs]
        outs = [torch.empty((Q.shape[0], lm.n_basis, lm.n_cells), dtype=tdt, device=dev)
                for lm, Q in zip(meshes, Qs)]
        alg = sum(algorithmic_bytes_per_cell(m.dim, M, lm.n_e, Q.shape[0], s) * m.n_cells
                  for (m, M, _), lm, Q in zip(raw, meshes, Qs))
        t0 = time.perf_counter()
        batch = C.Batch(meshes, [Q.shape[0] for Q in Qs], dtype=tag)
        t_batch = time.perf_counter() - t0
        ms_b = time_loop(torch, lambda: batch.run(qs, outs), steps, 3)
        for lm, q, o in zip(meshes, qs, outs):
            lm.tune(q, o, repeats=2)
        ms_m = time_loop(torch, lambda: [lm.reconstruct(q, out=o) for lm, q, o in zip(meshes, qs, outs)], steps, 2)
        info = batch.info()
        out[tag] = {
            "batch_graph_ms": ms_b, "batch_value": cv / (ms_b * 1e-3),
            "batch_roofline": dict(bound="hbm", achieved=alg / (ms_b * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                                   frac=alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, algorithmic_bytes=alg),
            "per_mesh_launches_ms": ms_m, "per_mesh_value": cv / (ms_m * 1e-3),
            "batch_create_s": t_batch, "groups": info["groups"]}
        log(f"batch {tag}: graph {ms_b:.3f} ms ({cv / (ms_b * 1e-3):.3e} cells*vars/s, "
            f"{100 * alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS:.1f}% of HBM peak); per-mesh launches {ms_m:.3f} ms")
        del batch, qs, outs
    out["f32_batch_vs_f64_per_mesh"] = out["f64"]["per_mesh_launches_ms"] / out["f32"]["batch_graph_ms"]
    return out


def serve_run(torch, srv, ids, qs, outs, cv, arrivals, picks):
    """Submit requests at their scheduled times; returns latency and throughput figures."""
    t0 = time.perf_counter() + 0.05
    tickets, lag = [], 0.0
    for a, k in zip(arrivals, picks):
        ts = t0 + a
        now = time.perf_counter()
        while now < ts:
            now = time.perf_counter()
        lag = max(lag, now - ts)
        tickets.append(srv.submit(ids[k], qs[k], outs[k]))
    for t in tickets:
        srv.wait(t, 600.0)
    wall = time.perf_counter() - t0
    st = srv.stats()
    served = sum(cv[k] for k in picks)
    return dict(requests=len(tickets), p50_ms=1e3 * st["p50_s"], p99_ms=1e3 * st["p99_s"],
                p999_ms=1e3 * st["p999_s"], evictions=st["evictions"], uploads=st["uploads"],
                upload_gb=st["upload_bytes"] / 1e9, wall_s=wall, value=served / wall,
                max_submit_lag_ms=1e3 * lag)


def measure_serving(torch, C, seconds, rate=2000.0, n_meshes=200, lo=2e3, hi=5e4, nv=5, budget_factor=1.54):
    """Registered meshes served from an HBM budget of budget_factor times their FP32
    footprint (the FP32 operators fit, the FP64 ones, twice as large, do not), Poisson
    arrivals; every mesh is requested once before the timed run."""
    from synthetic import batch_spec, workload_mesh
    spec = batch_spec(n_meshes, lo, hi, seed=16120938)
    t0 = time.perf_counter()
    raw = [(workload_mesh(d, n, sd), M) for d, n, M, sd in spec]
    hosts = [C.Mesh(m.vertices, m.cells, M, periodic=m.box, host_only=True) for m, M in raw]
    t_pre = time.perf_counter() - t0
    cells = sum(m.n_cells for m, _ in raw)
    cv = [m.n_cells * nv for m, _ in raw]
    rng = np.random.default_rng(16120939)
    n_req = int(seconds * rate)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    picks = [int(k) for k in rng.integers(0, n_meshes, size=n_req)]
    out = {"workload": f"{n_meshes} registered meshes, cell counts log-uniform on [{lo:.0e}, {hi:.0e}] ({cells} "
                       f"cells), d in {{2,3}}, M in {{2,3,4}}, {nv} variables; Poisson arrivals at {rate:.0f}/s, "
                       f"uniform mesh choice; HBM budget {budget_factor} x the FP32 operator footprint for both "
                       f"precisions (FP32 fits, FP64 needs evictions); every mesh requested once before timing",
           "cells": cells, "precompute_s": t_pre}
    probe = C.Server(64 << 30, dtype="f32")
    foot32 = sum(probe.mesh_info(probe.register_mesh(h))["image_bytes"] for h in hosts)
    del probe
    budget = int(budget_factor * foot32)
    log(f"serving: {n_meshes} meshes, {cells} cells, precompute {t_pre:.1f} s")
    for tag, tdt, inflight, streams, secs in (("f32", torch.float32, 16, 16, seconds),
                                              ("f64", torch.float64, 16, 16, min(seconds, 3.0)),
                                              ("f64_serial", torch.float64, 1, 1, min(seconds, 2.0))):
        dt = "f32" if tag == "f32" else "f64"
        srv = C.Server(budget, dtype=dt, max_inflight=inflight, n_streams=streams)
        ids = [srv.register_mesh(h) for h in hosts]
        qs = [torch.tensor(rng.normal(size=(nv, m.n_cells)), dtype=tdt, device="cuda:0") for m, _ in raw]
        outs = [torch.empty((nv, h.n_basis, h.n_cells), dtype=tdt, device="cuda:0") for h in hosts]
        torch.cuda.synchronize()
        # warm-up: every mesh once (what fits stays resident), then clean statistics
        foot = sum(srv.mesh_info(i)["image_bytes"] for i in ids)
        for k in range(n_meshes):
            srv.wait(srv.submit(ids[k], qs[k], outs[k]), 60.0)
        srv.reset_stats()
        n = int(secs * rate)
        r = serve_run(torch, srv, ids, qs, outs, cv, arrivals[:n], picks[:n])
        r.update(footprint_gb=foot / 1e9, budget_gb=budget / 1e9, max_inflight=inflight, streams=streams)
        out[tag] = r
        log(f"serving {tag}: {r['requests']} requests, p50 {r['p50_ms']:.3f} ms, p99 {r['p99_ms']:.3f} ms, "
            f"p99.9 {r['p999_ms']:.3f} ms, {r['value']:.3e} cells*vars/s, evictions {r['evictions']}")
        del srv, qs, outs
    return out


_ORACLE = None


def _oracle_worker_init(vertices, cells, box, Q, degree, factor):
    """Pool worker set-up: its own oracle of the benchmark mesh (no GPU)."""
    global _ORACLE
    from oracle import CwenoOracle, Options
    _ORACLE = (CwenoOracle(vertices, cells, box, Options(degree=degree, stencil_factor=factor)), Q)


def _oracle_worker_run(job):
    """Reconstruct cells of one block for about budget_s seconds on one thread."""
    from threadpoolctl import threadpool_limits
    block, budget_s = job
    o, Q = _ORACLE
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s and done < len(block):
            o.reconstruct_cell(int(block[done]), Q)
            done += 1
        dt = time.perf_counter() - t0
    return done, dt


def cpu_baseline(m, Q, degree, factor, budget_s, all_cores_s):
    """The CPU oracle on a bounded sample of the same workload's cells: one
    thread, then (all_cores_s > 0) a process pool of one single-threaded
    worker per available core over disjoint blocks of the sample."""
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
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0))
    out = dict(value=done * Q.shape[0] / dt, unit="cells·vars/s", cores=1, kind="oracle",
               sample=f"{done} random cells of the benchmark mesh (all {Q.shape[0]} variables), "
                      f"one thread, {dt:.1f} s; oracle set-up (face adjacency) excluded",
               host_cores_available=avail, cpu_model=model)
    nw = min(16, avail)
    if all_cores_s > 0 and nw > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        # spawned workers start from a fresh interpreter: nothing of this
        # process's GPU state is inherited, and none of them touches the GPU;
        # a worker that dies breaks the pool (an error here, never a hang)
        blocks = np.array_split(cells, nw)
        try:
            with ProcessPoolExecutor(nw, mp_context=mp.get_context("spawn"), initializer=_oracle_worker_init,
                                     initargs=(m.vertices, m.cells, m.box, Q, degree, factor)) as pool:
                res = list(pool.map(_oracle_worker_run, [(b, all_cores_s) for b in blocks]))
            total = sum(n for n, _ in res)
            out["all_cores"] = dict(
                value=sum(n / t for n, t in res) * Q.shape[0], unit="cells·vars/s", cores=nw, kind="oracle",
                sample=f"{total} cells in {nw} disjoint blocks of the same random order, one single-threaded "
                       f"process per block for {all_cores_s:.0f} s each (sum of the per-process rates); "
                       f"per-process oracle set-up excluded")
        except Exception as exc:              # reported, never fatal to the headline line
            out["all_cores"] = {"error": repr(exc)}
    return out


def measured_copy_gbs(torch):
    """Bandwidth of a plain 1 GiB device-to-device copy (bytes read + written per second)."""
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    ms = time_loop(torch, lambda: b.copy_(a), 20, 3)
    return 2 * a.numel() * 8 / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-all-cores-seconds", type=float, default=10.0,
                    help="length of the all-cores oracle run (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="only the main workload (and its moving-mesh form)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-mesh batch workload")
    ap.add_argument("--no-moving", action="store_true", help="skip the moving-mesh workloads")
    ap.add_argument("--no-weno", action="store_true", help="skip the classical WENO comparison")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the serving run (0 skips it)")
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
    from synthetic import kuhn_tet_mesh, tri_mesh, workload_fields

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    d, M, n, factor = 2, 3, 512, 0.0
    log("generating mesh and fields")
    m = tri_mesh(n, 0.15, SEED)
    Q = workload_fields(m, "mhd2d", SEED)
    nv = Q.shape[0]
    res = measure(torch, C, m, Q, M, factor, args.steps, args.warmup, "tri512 M3", d)
    copy_gbs = measured_copy_gbs(torch)
    log(f"plain device copy: {copy_gbs:.0f} GB/s")
    for tag in ("f64", "f32"):
        res[tag]["roofline"]["traffic"] = load_traffic(tag)
        res[tag]["roofline"]["measured_copy_gbs"] = copy_gbs
        res[tag]["roofline"]["frac_of_measured_copy"] = res[tag]["roofline"]["achieved"] / copy_gbs

    extras = {}
    try:
        extras["evaluate_tri512_M3_nv9"] = measure_evaluate(torch, C, res["mesh"], Q, M, d, 50)
    except Exception as exc:          # reported, never fatal to the headline line
        log(f"evaluate workload failed: {exc!r}")
        extras["evaluate_tri512_M3_nv9"] = {"error": repr(exc)}
    if not args.no_moving:
        try:
            stored2 = {tag: res[tag]["ms_per_step"] for tag in ("f64", "f32")}
            extras["moving_tri512_M3_nv9"] = measure_moving(torch, C, m, Q, M, "tri512 M3", d, 10, stored2)
        except Exception as exc:          # reported, never fatal to the headline line
            log(f"moving workload failed: {exc!r}")
            extras["moving_tri512_M3_nv9"] = {"error": repr(exc)}
    if not args.quick:
        if not args.no_weno:
            try:
                extras["weno_tri512_M3_nv9"] = measure_weno(torch, C, m, Q, M, d, 10, res["f64"]["ms_per_step"],
                                                            res["n_e"])
            except Exception as exc:          # reported, never fatal to the headline line
                log(f"weno workload failed: {exc!r}")
                extras["weno_tri512_M3_nv9"] = {"error": repr(exc)}
        # small mesh: launch-bound, reported as latency
        m1 = tri_mesh(64, 0.15, 16120934)
        Q1 = workload_fields(m1, "euler2d_sod", 16120934)
        r1 = measure(torch, C, m1, Q1, 2, 1.5, 200, 20, "tri64 M2", 2)
        extras["tri64_M2_nv4"] = {
            "workload": "2-D M=2, 8,192 jittered periodic triangles, n_e=9 (stencil factor 1.5), 4 Euler variables",
            "f64_latency_ms": r1["f64"]["latency_ms"], "f32_latency_ms": r1["f32"]["latency_ms"],
            "f64_value": r1["f64"]["value"], "f32_value": r1["f32"]["value"], "unit": "cells·vars/s"}
        del r1
        # 3-D throughput
        m3 = kuhn_tet_mesh(64, 0.1, 16120936)
        Q3 = workload_fields(m3, "euler3d_blast", 16120936)
        r3 = measure(torch, C, m3, Q3, 3, 0.0, 20, 3, "kuhn64 M3", 3)
        extras["kuhn64_M3_nv5"] = {
            "workload": "3-D M=3, 1,572,864 jittered periodic Kuhn tetrahedra, n_e=60, 4 sectors, 5 variables",
            "precompute_s": r3["precompute_s"],
            "precompute_device_operators_s": r3.get("precompute_device_operators_s")}
        for tag in ("f64", "f32"):
            extras["kuhn64_M3_nv5"][tag] = {k: r3[tag][k] for k in ("value", "ms_per_step", "latency_ms", "roofline",
                                                                   "variant", "flushed_ms", "flushed_frac")}
        stored3 = {tag: r3[tag]["ms_per_step"] for tag in ("f64", "f32")}
        del r3
        if not args.no_moving:
            try:
                extras["moving_kuhn64_M3_nv5"] = measure_moving(torch, C, m3, Q3, 3, "kuhn64 M3", 3, 5, stored3)
            except Exception as exc:          # reported, never fatal to the headline line
                log(f"moving workload failed: {exc!r}")
                extras["moving_kuhn64_M3_nv5"] = {"error": repr(exc)}
        del m3, Q3
        if not args.no_batch:
            try:
                extras["batch64_mixed"] = measure_batch(torch, C, 20)
            except Exception as exc:          # reported, never fatal to the headline line
                log(f"batch workload failed: {exc!r}")
                extras["batch64_mixed"] = {"error": repr(exc)}
        if args.serve_seconds > 0:
            try:
                extras["serving"] = measure_serving(torch, C, args.serve_seconds)
            except Exception as exc:          # reported, never fatal to the headline line
                log(f"serving workload failed: {exc!r}")
                extras["serving"] = {"error": repr(exc)}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(m, Q, M, factor, args.cpu_seconds, args.cpu_all_cores_seconds)
        log(f"cpu: {cpu['value']:.3e} cells*vars/s on one thread"
            + (f", {cpu['all_cores']['value']:.3e} on {cpu['all_cores']['cores']} processes"
               if "value" in cpu.get("all_cores", {}) else ""))

    r64 = res["f64"]
    line = {
        "metric": METRIC, "value": r64["value"], "unit": "cells·vars/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "CWENO 2-D M=3 (10 basis functions), 524,288 jittered periodic triangles "
                               "(512x512x2), n_e=20, 3 sectors, 9 MHD-shaped variables",
                   "cells": m.n_cells, "n_vars": nv, "degree": M, "dim": d, "n_e": res["n_e"],
                   "lambda0": 0.95, "eps": 1e-14, "r": 4, "seed": SEED},
        "roofline": r64["roofline"],
        "latency_ms": r64["latency_ms"],
        "cache_flushed": {"f64_ms": r64["flushed_ms"], "f64_frac": r64["flushed_frac"],
                          "f32_ms": res["f32"]["flushed_ms"], "f32_frac": res["f32"]["flushed_frac"],
                          "note": "median single launch after a 1 GiB overwrite; value and roofline are "
                                  "back-to-back launches"},
        "kernel_variant": {"f64": res["f64"]["variant"], "f32": res["f32"]["variant"]},
        "fp32": {"value": res["f32"]["value"], "ms_per_step": res["f32"]["ms_per_step"],
                 "latency_ms": res["f32"]["latency_ms"], "roofline": res["f32"]["roofline"],
                 "dtype": "f32"},
        "cpu_baseline": cpu,
        "precompute_s": res["precompute_s"],
        "precompute_device_operators_s": res.get("precompute_device_operators_s"),
        "extras": extras,
        "kernel_source_sha": kernel_source_hash(),
        "moving_kernel_source_sha": kernel_source_hash(MOVING_SRCS),
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
