"""Benchmark: CWENO reconstruction throughput on one MI355X.

Headline workload: 3-D, degree M = 3 (20 basis functions), 64^3 cubes x 6 =
1,572,864 jittered periodic Kuhn tetrahedra, central stencil n_e = 60,
4 cone sectors, 5 Euler variables (spherical blast plus a smooth
perturbation).  One step = one cweno_reconstruct of the whole mesh (all
five steps of the method for every cell and variable), inputs already
resident in HBM.

Prints one JSON line.  ``value`` is the FP64 path's cells*vars/s; the FP32
operator path is reported beside it under "fp32".  The other workloads go
under "extras" (``--only`` picks a subset by name):

* tri512   -- 2-D M=3, 524,288 jittered periodic triangles, 9 MHD-shaped
              variables, both precisions (and its cache-flushed launch);
* tri64    -- 2-D M=2, 8,192 triangles, 4 Euler variables: launch latency;
* evaluate -- point values of the tri512 reconstruction at face Gauss points,
              separate and fused;
* moving2d, moving3d -- the moving-mesh form (operators rebuilt from the
              vertices in every call) on the tri512 and headline meshes;
* weno     -- the classical unstructured WENO scheme on the tri512 workload;
* batch    -- 64 uneven meshes of mixed dimension and degree in one graph;
* serving  -- registered meshes under an HBM budget, Poisson arrivals.

The CPU oracle is timed on a bounded sample of the headline workload
(``cpu_baseline``); the same oracle cells, and bounded samples of the other
reconstruction workloads, give the FP64 and FP32 errors against the oracle
per workload (``oracle_error``).
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
SEED = 16120935                 # 2-D M=3, 524,288 triangles
SEED1 = 16120934                # 2-D M=2, 8,192 triangles
SEED3 = 16120936                # 3-D M=3, 1,572,864 tetrahedra
CSRC = os.path.join(ROOT, "paper_1612_09335_amd", "csrc")
KERNEL_SRCS = ["reconstruct_kernel.hpp", "halo_kernel.hpp", "dispatch.hpp", "kernels.hip", "gen_sigma.cpp"]
MOVING_SRCS = ["moving_kernel.hpp", "moving.hpp", "moving_kernels.hip"]
WENO_SRCS = ["weno.hip", "weno.hpp"]
EVAL_SRCS = ["evaluate.hip"]
BATCH_SRCS = KERNEL_SRCS + ["batch.hip"]
WORKLOADS = ("kuhn64", "tri512", "tri64", "evaluate", "moving2d", "moving3d", "weno", "batch", "serving")


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
    stored_ms = stored_ms or {}
    out = {"workload": f"{label} with every vertex moved (smooth periodic shear, gradient 0.2); stencils of the "
                       f"connectivity, operators rebuilt per call", "registration_s": t_reg,
           "device_bytes": lm.device_bytes, "flops_per_launch": flops}
    fault = torch.zeros(1, dtype=torch.int32, device=dev)
    for tag, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        q = torch.tensor(Q, dtype=tdt, device=dev)
        o = torch.empty((nv, lm.n_basis, lm.n_cells), dtype=tdt, device=dev)
        ms = time_loop(torch, lambda: lm.reconstruct_moving(V, q, out=o, fault=fault), steps, 2)
        tf = flops / (ms * 1e-3) / 1e12
        ratio = ms / stored_ms[tag] if tag in stored_ms else None
        out[tag] = {"ms_per_step": ms, "value": m.n_cells * nv / (ms * 1e-3),
                    "vs_stored_operators": ratio,
                    "roofline": dict(bound="alu", achieved=tf, peak=FP64_VECTOR_TFS, unit="TFLOP/s",
                                     frac=tf / FP64_VECTOR_TFS,
                                     traffic=load_traffic(("moving_" if d == 2 else "moving3d_") + tag,
                                                          MOVING_SRCS))}
        log(f"moving {label} {tag}: {ms:.3f} ms ({out[tag]['value']:.3e} cells*vars/s, {tf:.2f} TFLOP/s FP64"
            + (f", {ratio:.1f}x the stored-operator launch)" if ratio else ")"))
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
                                     frac=gbs / HBM_PEAK_GBS, traffic=load_traffic("evaluate_" + tag, EVAL_SRCS),
                                     algorithmic_bytes_per_launch=alg),
                    "reconstruct_then_evaluate_ms": ms_two, "fused_ms": ms_fused,
                    "fused_roofline": dict(bound="hbm", achieved=fused_alg / (ms_fused * 1e-3) / 1e9,
                                           peak=HBM_PEAK_GBS, unit="GB/s",
                                           frac=fused_alg / (ms_fused * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                           traffic=load_traffic("fused_points_" + tag),
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
         "algorithmic_byte_ratio_weno_over_cweno":
             alg / (algorithmic_bytes_per_cell(d, M, cweno_n_e, nv, 8) * m.n_cells),
         "ms_per_step": ms, "steps": steps, "value": m.n_cells * nv / (ms * 1e-3),
         "time_ratio_weno_over_cweno_f64": ms / cweno_ms, "operator_passes": passes,
         "comparison_note": "the algorithmic byte ratio is the schemes' comparison at equal streaming rates; "
                            "the time ratio also holds the two kernels' different fractions of HBM peak "
                            "(implementation-limited)",
         "roofline": dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                          traffic=load_traffic("weno_f64", WENO_SRCS), algorithmic_bytes_per_launch=alg,
                          streamed_bytes_per_launch=streamed,
                          streamed_frac=streamed / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)}
    log(f"weno: precompute {t_pre:.1f} s, {lm.device_bytes / 1e9:.2f} GB on the device, {ms:.3f} ms "
        f"({ms / cweno_ms:.1f}x CWENO FP64; algorithmic bytes "
        f"{r['algorithmic_byte_ratio_weno_over_cweno']:.2f}x), operators {weno_entries / cweno_entries:.2f}x CWENO's "
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
    """Per-launch ms after a read-only pass over 1 GiB between launches: the
    256 MB Infinity Cache and the L2s then hold none of the operators when a
    launch starts, and as the flush only reads, the timed launch inherits no
    dirty lines to write back (the previous launch's coefficients are written
    back during the flush)."""
    flush.fill_(1.0)
    sink = torch.empty((), dtype=flush.dtype, device=flush.device)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        sink.copy_(flush.sum())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mesh.reconstruct(q, out=out)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times))


def measure(torch, C, m, Q, M, factor, steps, warmup, label, d, keep_out=False):
    """Time both precisions on one workload; returns per-precision records
    (with keep_out, also each precision's coefficients as a host array under
    "out", for the comparison with the oracle)."""
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
        if keep_out:
            res[tag]["out"] = r["out"].cpu().numpy()
        del r
        log(f"{label} {tag}: variant {res[tag]['variant']}, {ms:.4f} ms/step, {res[tag]['value']:.3e} cells*vars/s, "
            f"{achieved:.0f} GB/s ({100 * achieved / HBM_PEAK_GBS:.1f}% of peak); cache-flushed launch "
            f"{ms_flushed:.4f} ms ({100 * res[tag]['flushed_frac']:.1f}%)")
    return res


WARM_S = 0.1


def time_loop(torch, fn, steps, warmup):
    """Average ms of fn() over `steps` back-to-back calls on the current stream,
    after at least `warmup` calls and at least WARM_S seconds of back-to-back
    calls: the GPU idles while the host builds a workload, and the launches
    right after such a pause run slower (those of a 1.4 ms kernel fell from
    1.8 ms to 1.37 ms over the first 20, most likely while the clocks come
    back up from idle)."""
    t0 = time.perf_counter()
    while True:
        for _ in range(max(warmup, 1)):
            fn()
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= WARM_S:
            break
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def measure_batch(torch, C, steps, oracle_cells_per_mesh=16):
    """64 uneven meshes (seeded recipe): FP32 batch graph vs per-mesh launches,
    and both precisions' coefficients on a seeded sample of every mesh's cells
    against the oracle."""
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
    rng = np.random.default_rng(SEED + 4)
    picks = [np.sort(rng.choice(m.n_cells, size=min(oracle_cells_per_mesh, m.n_cells), replace=False))
             for m, _, _ in raw]
    sampled = {}
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
        sampled[tag] = [o[:, :, torch.as_tensor(c, device=dev)].cpu().numpy() for o, c in zip(outs, picks)]
        for lm, q, o in zip(meshes, qs, outs):
            lm.tune(q, o, repeats=2)
        ms_m = time_loop(torch, lambda: [lm.reconstruct(q, out=o) for lm, q, o in zip(meshes, qs, outs)], steps, 2)
        info = batch.info()
        out[tag] = {
            "batch_graph_ms": ms_b, "batch_value": cv / (ms_b * 1e-3),
            "batch_roofline": dict(bound="hbm", achieved=alg / (ms_b * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                                   frac=alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, algorithmic_bytes=alg,
                                   traffic=load_traffic("batch_" + tag, BATCH_SRCS)),
            "per_mesh_launches_ms": ms_m, "per_mesh_value": cv / (ms_m * 1e-3),
            "batch_create_s": t_batch, "groups": info["groups"]}
        log(f"batch {tag}: graph {ms_b:.3f} ms ({cv / (ms_b * 1e-3):.3e} cells*vars/s, "
            f"{100 * alg / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS:.1f}% of HBM peak); per-mesh launches {ms_m:.3f} ms")
        del batch, qs, outs
    out["f32_batch_vs_f64_per_mesh"] = out["f64"]["per_mesh_launches_ms"] / out["f32"]["batch_graph_ms"]
    # the oracle on the sampled cells of every mesh (FP32: the batch graph's
    # output; FP64: the per-mesh launches')
    t0 = time.perf_counter()
    jobs = [(m.vertices, m.cells, m.box, Q, M, 0.0, c) for (m, M, _), Q, c in zip(raw, Qs, picks)]
    parts = oracle_pool(host_workers(), _oracle_mesh_job, jobs)
    per = {"f64": [], "f32": []}
    for k, prt in enumerate(parts):
        prt = dict(prt, cells=np.arange(len(picks[k])))          # columns of the sampled arrays
        for t in per:
            per[t].append(per_cell_error([prt], sampled[t][k]))
    out["oracle_error"] = error_summary({t: np.concatenate(v) for t, v in per.items()},
                                        f"{oracle_cells_per_mesh} seeded random cells of each of the "
                                        f"{len(raw)} meshes")
    out["oracle_error"]["oracle_s"] = time.perf_counter() - t0
    log(f"batch oracle error: FP32 max {out['oracle_error']['f32_max']:.2e}, FP64 max "
        f"{out['oracle_error']['f64_max']:.2e} over {out['oracle_error']['cells_compared']} cells")
    return out


def serve_run(torch, srv, ids, qs, outs, cv, arrivals, picks):
    """Submit requests at their scheduled times; returns latency and throughput figures."""
    srv.reset_stats()
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
    st, ls = srv.stats(), srv.launch_stats()
    served = sum(cv[k] for k in picks)
    return dict(requests=len(tickets), rate_per_s=len(tickets) / float(arrivals[-1]) if len(arrivals) else 0.0,
                p50_ms=1e3 * st["p50_s"], p99_ms=1e3 * st["p99_s"],
                p999_ms=1e3 * st["p999_s"], evictions=st["evictions"], uploads=st["uploads"],
                upload_gb=st["upload_bytes"] / 1e9, wall_s=wall, value=served / wall,
                max_submit_lag_ms=1e3 * lag, launches=ls["launches"], shared_requests=ls["shared_requests"],
                largest_launch=ls["largest_launch"])


def measure_serving(torch, C, seconds, rate=2000.0, n_meshes=200, lo=2e3, hi=5e4, nv=5, budget_factor=1.54,
                    sweep=(2000.0, 8000.0, 32000.0, 128000.0), sweep_seconds=2.0):
    """Registered meshes served from an HBM budget of budget_factor times their FP32
    footprint (the FP32 operators fit, the FP64 ones, twice as large, do not), Poisson
    arrivals; every mesh is requested once before the timed runs.  FP32 at the
    nominal rate with requests batched as they arrive, then a sweep of arrival
    rates with and without batching; FP64 (evicting), a serial FP64 server, and
    FP64 under a budget of 1.1 times its own footprint (resident)."""
    from synthetic import batch_spec, workload_mesh
    spec = batch_spec(n_meshes, lo, hi, seed=16120938)
    t0 = time.perf_counter()
    raw = [(workload_mesh(d, n, sd), M) for d, n, M, sd in spec]
    hosts = [C.Mesh(m.vertices, m.cells, M, periodic=m.box, host_only=True) for m, M in raw]
    t_pre = time.perf_counter() - t0
    cells = sum(m.n_cells for m, _ in raw)
    cv = [m.n_cells * nv for m, _ in raw]
    rng = np.random.default_rng(16120939)
    gaps = rng.exponential(1.0, size=int(max(seconds, sweep_seconds) * max((rate,) + tuple(sweep))) + 1)
    picks = [int(k) for k in rng.integers(0, n_meshes, size=len(gaps))]

    def arrivals(r, secs):
        n = int(secs * r)
        return np.cumsum(gaps[:n]) / r, picks[:n]

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

    def server(dt, tdt, inflight, streams, batch, budget_bytes=None):
        srv = C.Server(budget_bytes or budget, dtype=dt, max_inflight=inflight, n_streams=streams, max_batch=batch)
        ids = [srv.register_mesh(h) for h in hosts]
        qs = [torch.tensor(rng.normal(size=(nv, m.n_cells)), dtype=tdt, device="cuda:0") for m, _ in raw]
        outs = [torch.empty((nv, h.n_basis, h.n_cells), dtype=tdt, device="cuda:0") for h in hosts]
        torch.cuda.synchronize()
        # warm-up: every mesh once (what fits stays resident)
        for k in range(n_meshes):
            srv.wait(srv.submit(ids[k], qs[k], outs[k]), 60.0)
        return srv, ids, qs, outs

    def report(tag, r):
        log(f"serving {tag}: {r['requests']} requests at {r['rate_per_s']:.0f}/s, p50 {r['p50_ms']:.3f} ms, "
            f"p99 {r['p99_ms']:.3f} ms, p99.9 {r['p999_ms']:.3f} ms, {r['value']:.3e} cells*vars/s, "
            f"{r['launches']} launches (largest {r['largest_launch']}), evictions {r['evictions']}")

    # FP32, operators resident: nominal rate, then the sweep with and without batching
    srv, ids, qs, outs = server("f32", torch.float32, 8, 8, 64)
    foot = sum(srv.mesh_info(i)["image_bytes"] for i in ids)
    r = serve_run(torch, srv, ids, qs, outs, cv, *arrivals(rate, seconds))
    r.update(footprint_gb=foot / 1e9, budget_gb=budget / 1e9, max_inflight=8, streams=8, max_batch=64)
    out["f32"] = r
    report("f32", r)
    out["f32_sweep"] = []
    for rr in sweep:
        for batch in (64, 1):
            srv.set_batch(batch)
            r = serve_run(torch, srv, ids, qs, outs, cv, *arrivals(rr, sweep_seconds))
            r.update(max_batch=batch)
            out["f32_sweep"].append(r)
            report(f"f32 sweep batch {batch}", r)
    del srv, qs, outs
    for tag, inflight, streams, batch, secs in (("f64", 8, 8, 64, min(seconds, 3.0)),
                                                ("f64_serial", 1, 1, 1, min(seconds, 2.0))):
        srv, ids, qs, outs = server("f64", torch.float64, inflight, streams, batch)
        foot = sum(srv.mesh_info(i)["image_bytes"] for i in ids)
        r = serve_run(torch, srv, ids, qs, outs, cv, *arrivals(rate, secs))
        r.update(footprint_gb=foot / 1e9, budget_gb=budget / 1e9, max_inflight=inflight, streams=streams,
                 max_batch=batch)
        out[tag] = r
        report(tag, r)
        del srv, qs, outs
    # FP64 under a budget that holds every image: the FP64 served rate without eviction
    b64 = int(1.1 * out["f64"]["footprint_gb"] * 1e9)
    srv, ids, qs, outs = server("f64", torch.float64, 8, 8, 64, b64)
    r = serve_run(torch, srv, ids, qs, outs, cv, *arrivals(rate, min(seconds, 3.0)))
    r.update(footprint_gb=out["f64"]["footprint_gb"], budget_gb=b64 / 1e9, max_inflight=8, streams=8, max_batch=64)
    out["f64_resident"] = r
    report("f64 resident", r)
    del srv, qs, outs
    return out


def measure_serving_full(torch, C, seconds, rate=2000.0, n_meshes=200, lo=2e3, hi=1e6, nv=5, budget_gb=200.0,
                         sweep=(2000.0, 8000.0, 32000.0), sweep_seconds=3.0, oracle_meshes=4):
    """The served configuration at its stated scale: 200 meshes of 2k-1M cells
    (log-uniform), FP32 operators under a 200 GB HBM budget, Poisson arrivals.
    Each mesh is registered right after its host precompute (the server keeps
    only its pinned FP32 image), so host memory holds the FP32 images (about
    140 GB) and one mesh's FP64 operators at a time.  The FP64 images (about
    270 GB) do not fit the host memory one process may use here, so there is no
    FP64 server at this scale.  Sampled cells of served results on a few small
    meshes are compared with the oracle."""
    from synthetic import batch_spec, workload_mesh
    spec = batch_spec(n_meshes, lo, hi, seed=16120938)
    srv = C.Server(int(budget_gb * 1e9), dtype="f32", max_inflight=8, n_streams=8, max_batch=64)
    t0 = time.perf_counter()
    raw, ids, foot = [], [], 0
    for k, (d, n, M, sd) in enumerate(spec):
        m = workload_mesh(d, n, sd)
        ids.append(srv.register(m.vertices, m.cells, M, periodic=m.box))
        info = srv.mesh_info(ids[-1])
        foot += info["image_bytes"]
        raw.append((m if m.n_cells <= 60000 else None, d, M, m.n_cells, info["n_basis"]))
        log(f"serving full: registered {k + 1} meshes ({d}-D, M={M}, {m.n_cells} cells), "
            f"{sum(r[3] for r in raw)} cells, {foot / 1e9:.1f} GB of FP32 images, {time.perf_counter() - t0:.0f} s")
    t_reg = time.perf_counter() - t0
    cells = sum(r[3] for r in raw)
    cv = [r[3] * nv for r in raw]
    rng = np.random.default_rng(16120939)
    qs = [torch.tensor(rng.normal(size=(nv, r[3])), dtype=torch.float32, device="cuda:0") for r in raw]
    outs = [torch.empty((nv, r[4], r[3]), dtype=torch.float32, device="cuda:0") for r in raw]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_meshes):                      # warm-up: every mesh once
        srv.wait(srv.submit(ids[k], qs[k], outs[k]), 120.0)
    t_warm = time.perf_counter() - t0
    st = srv.stats()
    out = {"workload": f"{n_meshes} registered meshes, cell counts log-uniform on [{lo:.0e}, {hi:.0e}] ({cells} "
                       f"cells), d in {{2,3}}, M in {{2,3,4}}, {nv} variables, FP32 operators under an HBM budget of "
                       f"{budget_gb:.0f} GB; Poisson arrivals, uniform mesh choice; every mesh requested once "
                       f"before timing",
           "cells": cells, "registration_s": t_reg, "fp32_footprint_gb": foot / 1e9, "budget_gb": budget_gb,
           "warmup_s": t_warm, "warmup_uploads": st["uploads"], "warmup_upload_gb": st["upload_bytes"] / 1e9,
           "fp64": "not measured at this scale: the FP64 images (about twice the FP32 footprint) exceed the host "
                   "memory one process may use on the benchmark host"}
    gaps = rng.exponential(1.0, size=int(max(seconds, sweep_seconds) * max((rate,) + tuple(sweep))) + 1)
    picks = [int(k) for k in rng.integers(0, n_meshes, size=len(gaps))]

    def arrivals(r, secs):
        n = int(secs * r)
        return np.cumsum(gaps[:n]) / r, picks[:n]

    def report(tag, r):
        log(f"serving full {tag}: {r['requests']} requests at {r['rate_per_s']:.0f}/s, p50 {r['p50_ms']:.3f} ms, "
            f"p99 {r['p99_ms']:.3f} ms, p99.9 {r['p999_ms']:.3f} ms, {r['value']:.3e} cells*vars/s, "
            f"{r['launches']} launches (largest {r['largest_launch']}), evictions {r['evictions']}")

    r = serve_run(torch, srv, ids, qs, outs, cv, *arrivals(rate, seconds))
    out["f32"] = r
    report("f32", r)
    out["f32_sweep"] = []
    for rr in sweep:
        for batch in (64, 1):
            srv.set_batch(batch)
            r = serve_run(torch, srv, ids, qs, outs, cv, *arrivals(rr, sweep_seconds))
            r.update(max_batch=batch)
            out["f32_sweep"].append(r)
            report(f"sweep batch {batch}", r)
    srv.set_batch(64)
    # served results against the oracle: sampled cells of the smallest meshes
    small = sorted((k for k, rec in enumerate(raw) if rec[0] is not None), key=lambda k: raw[k][3])
    pick_d = [k for k in small if raw[k][1] == 2][:oracle_meshes // 2] + \
        [k for k in small if raw[k][1] == 3][:oracle_meshes - oracle_meshes // 2]
    errs = []
    Qo = {}
    for k in pick_d:
        m = raw[k][0]
        Q = np.random.default_rng(SEED + k).normal(size=(nv, m.n_cells))
        Qo[k] = Q
        q = torch.tensor(Q, dtype=torch.float32, device="cuda:0")
        o = torch.empty((nv, raw[k][4], m.n_cells), dtype=torch.float32, device="cuda:0")
        srv.wait(srv.submit(ids[k], q, o), 120.0)
        cells_k = np.sort(np.random.default_rng(SEED + 100 + k).choice(m.n_cells, size=32, replace=False))
        parts = oracle_pool(host_workers(), _oracle_mesh_job,
                            [(m.vertices, m.cells, m.box, Q, raw[k][2], 0.0, cells_k)])
        errs.append(per_cell_error(parts, o.cpu().numpy()))
    if errs:
        out["oracle_error"] = error_summary({"f32": np.concatenate(errs)},
                                            f"32 seeded cells of each of {len(errs)} served meshes "
                                            f"(the smallest 2-D and 3-D ones)")
        log(f"serving full: FP32 served results against the oracle, max {out['oracle_error']['f32_max']:.2e}")
    del srv, qs, outs
    return out


_ORACLE = None


def _oracle_cells(o, Q, ids, budget_s):
    """The oracle on cells ids (in order) for at most budget_s seconds, one
    thread: (cells done, seconds, their coefficients [k, nv, nb] and the data
    scale max over the central stencil of |Q| [k, nv])."""
    from threadpoolctl import threadpool_limits
    co, sc = [], []
    done = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while done < len(ids) and (budget_s is None or time.perf_counter() - t0 < budget_s):
            r = o.reconstruct_cell(int(ids[done]), Q)
            co.append(r["coeffs"])
            sc.append(np.abs(Q[:, r["stencil"]]).max(axis=1))
            done += 1
        dt = time.perf_counter() - t0
    nv, nb = Q.shape[0], o.nb
    return dict(done=done, seconds=dt, cells=np.asarray(ids[:done], dtype=np.int64),
                coeffs=np.array(co).reshape(done, nv, nb), scale=np.array(sc).reshape(done, nv))


def _oracle_worker_init(vertices, cells, box, Q, degree, factor):
    """Pool worker set-up: its own oracle of one mesh (no GPU)."""
    global _ORACLE
    from oracle import CwenoOracle, Options
    _ORACLE = (CwenoOracle(vertices, cells, box, Options(degree=degree, stencil_factor=factor)), Q)


def _oracle_worker_run(job):
    """Cells of one block of the pool's mesh, for at most budget_s seconds."""
    ids, budget_s = job
    o, Q = _ORACLE
    return _oracle_cells(o, Q, ids, budget_s)


def _oracle_mesh_job(job):
    """Cells ids of a mesh passed with the job (its own oracle, no time limit)."""
    from oracle import CwenoOracle, Options
    vertices, cells, box, Q, degree, factor, ids = job
    o = CwenoOracle(vertices, cells, box, Options(degree=degree, stencil_factor=factor))
    return _oracle_cells(o, Q, ids, None)


def oracle_pool(n_workers, fn, jobs, initargs=None):
    """Run fn over jobs in n_workers spawned single-threaded processes.

    Spawned workers start from a fresh interpreter: nothing of this process's
    GPU state is inherited and none of them touches the GPU.  The pool is shut
    down and its workers joined before returning, and so is multiprocessing's
    resource-tracker process, so that no child outlives the benchmark."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    kw = dict(mp_context=mp.get_context("spawn"))
    if initargs is not None:
        kw.update(initializer=_oracle_worker_init, initargs=initargs)
    try:
        with ProcessPoolExecutor(n_workers, **kw) as pool:
            return list(pool.map(fn, jobs))
    finally:
        try:
            from multiprocessing import resource_tracker
            resource_tracker._resource_tracker._stop()
        except Exception:
            pass


def host_workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def per_cell_error(parts, got):
    """Per cell, max over (v, l) of |got - oracle| / scale[v] (the data-scaled
    error): parts are oracle results (cells, coeffs [k, nv, nb], scale
    [k, nv]); got [nv, nb, n] is the library's output."""
    cells = np.concatenate([p["cells"] for p in parts])
    want = np.concatenate([p["coeffs"] for p in parts]).transpose(1, 2, 0)      # [nv, nb, k]
    scale = np.maximum(np.concatenate([p["scale"] for p in parts]).T, 1e-300)  # [nv, k]
    g = got[:, :, cells].astype(np.float64)
    return (np.abs(g - want) / scale[:, None, :]).max(axis=(0, 1))


def error_summary(per_cell, workload):
    """FP64: the largest error; FP32: the largest and the 99.9th percentile over cells."""
    r = {"workload": workload}
    for tag, e in per_cell.items():
        r["cells_compared"] = int(len(e))
        r[f"{tag}_max"] = float(e.max())
        r[f"{tag}_p999"] = float(np.percentile(e, 99.9))
    return r


def oracle_error(parts, outs, workload):
    """error_summary of the library's outputs {"f64": [nv, nb, n], "f32": ...} against the oracle."""
    return error_summary({tag: per_cell_error(parts, got) for tag, got in outs.items()}, workload)


def cpu_baseline(m, Q, degree, factor, budget_s, all_cores_s):
    """The CPU oracle on a bounded sample of the same workload's cells: one
    thread, then (all_cores_s > 0) a process pool of one single-threaded
    worker per available core over disjoint blocks of the sample.  Returns the
    record and the oracle results of every cell it reconstructed."""
    from oracle import CwenoOracle, Options
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=degree, stencil_factor=factor))
    rng = np.random.default_rng(SEED)
    cells = rng.permutation(m.n_cells)
    one = _oracle_cells(o, Q, cells, budget_s)
    done, dt = one["done"], one["seconds"]
    parts = [one]
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
    nw = host_workers()
    if all_cores_s > 0 and nw > 1:
        # the pool's blocks start after the cells the single thread did
        blocks = np.array_split(cells[done:], nw)
        try:
            res = oracle_pool(nw, _oracle_worker_run, [(b, all_cores_s) for b in blocks],
                              initargs=(m.vertices, m.cells, m.box, Q, degree, factor))
            total = sum(r["done"] for r in res)
            parts += res
            out["all_cores"] = dict(
                value=sum(r["done"] / r["seconds"] for r in res) * Q.shape[0], unit="cells·vars/s", cores=nw,
                kind="oracle",
                sample=f"{total} cells in {nw} disjoint blocks of the same random order, one single-threaded "
                       f"process per block for {all_cores_s:.0f} s each (sum of the per-process rates); "
                       f"per-process oracle set-up excluded")
        except Exception as exc:              # reported, never fatal to the headline line
            out["all_cores"] = {"error": repr(exc)}
    return out, parts


def oracle_sample(m, Q, degree, factor, cells):
    """Oracle results of the given cells of one mesh, over the host's cores."""
    nw = host_workers()
    blocks = [b for b in np.array_split(np.asarray(cells), nw) if len(b)]
    return oracle_pool(len(blocks), _oracle_worker_run, [(b, None) for b in blocks],
                       initargs=(m.vertices, m.cells, m.box, Q, degree, factor))


def measured_copy_gbs(torch):
    """Bandwidth of a plain 1 GiB device-to-device copy (bytes read + written per second)."""
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    ms = time_loop(torch, lambda: b.copy_(a), 20, 3)
    return 2 * a.numel() * 8 / (ms * 1e-3) / 1e9


def guarded(extras, key, fn):
    """extras[key] = fn(); a failure is reported there, never fatal to the headline line."""
    try:
        extras[key] = fn()
    except Exception as exc:
        log(f"{key} failed: {exc!r}")
        extras[key] = {"error": repr(exc)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-all-cores-seconds", type=float, default=10.0,
                    help="length of the all-cores oracle run (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the comparison of sampled cells with the oracle")
    ap.add_argument("--only", default=",".join(WORKLOADS),
                    help="comma-separated workloads to measure: " + ",".join(WORKLOADS))
    ap.add_argument("--serve-full", action="store_true",
                    help="serve the 200-mesh set at its stated scale (2k-1M cells, 200 GB budget; minutes of "
                         "registration) instead of the scaled set")
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
    only = set(w.strip() for w in args.only.split(",") if w.strip())
    unknown = only - set(WORKLOADS)
    if unknown:
        print(f"unknown workloads {sorted(unknown)}; choose from {','.join(WORKLOADS)}", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_09335_amd as C
    from synthetic import kuhn_tet_mesh, tri_mesh, workload_fields

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    errors = {}
    extras = {}
    copy_gbs = measured_copy_gbs(torch)
    log(f"plain device copy: {copy_gbs:.0f} GB/s")

    def with_traffic(rec, tag, key):
        rec["roofline"]["traffic"] = load_traffic(key)
        rec["roofline"]["measured_copy_gbs"] = copy_gbs
        rec["roofline"]["frac_of_measured_copy"] = rec["roofline"]["achieved"] / copy_gbs

    # headline: 3-D M=3 Kuhn tetrahedra, 5 Euler variables
    res3 = m3 = Q3 = None
    if "kuhn64" in only or "moving3d" in only:
        log("generating the 3-D mesh and fields")
        m3 = kuhn_tet_mesh(64, 0.1, SEED3)
        Q3 = workload_fields(m3, "euler3d_blast", SEED3)
    if "kuhn64" in only:
        res3 = measure(torch, C, m3, Q3, 3, 0.0, args.steps, args.warmup, "kuhn64 M3", 3,
                       keep_out=not args.no_oracle_error)
        for tag in ("f64", "f32"):
            with_traffic(res3[tag], tag, "kuhn64_M3_nv5_" + tag)
    if "moving3d" in only:
        stored3 = {tag: res3[tag]["ms_per_step"] for tag in ("f64", "f32")} if res3 else None
        guarded(extras, "moving_kuhn64_M3_nv5", lambda: measure_moving(torch, C, m3, Q3, 3, "kuhn64 M3", 3, 5,
                                                                       stored3))
    if res3 is not None:
        res3.pop("mesh", None)            # its 25 GB of operators are not needed again

    # 2-D M=3, 524,288 triangles, 9 MHD-shaped variables
    need2 = {"tri512", "evaluate", "moving2d", "weno"} & only
    m2 = Q2 = res2 = None
    if need2:
        log("generating the 2-D mesh and fields")
        m2 = tri_mesh(512, 0.15, SEED)
        Q2 = workload_fields(m2, "mhd2d", SEED)
        res2 = measure(torch, C, m2, Q2, 3, 0.0, args.steps, args.warmup, "tri512 M3", 2,
                       keep_out="tri512" in only and not args.no_oracle_error)
        for tag in ("f64", "f32"):
            with_traffic(res2[tag], tag, "tri512_M3_nv9_" + tag)
        if "tri512" in only:
            extras["tri512_M3_nv9"] = {
                "workload": "2-D M=3 (10 basis functions), 524,288 jittered periodic triangles (512x512x2), n_e=20, "
                            "3 sectors, 9 MHD-shaped variables",
                "precompute_s": res2["precompute_s"],
                "precompute_device_operators_s": res2.get("precompute_device_operators_s")}
            for tag in ("f64", "f32"):
                extras["tri512_M3_nv9"][tag] = {k: res2[tag][k] for k in (
                    "value", "ms_per_step", "kernel_ms", "latency_ms", "roofline", "variant", "flushed_ms",
                    "flushed_frac")}
    if "evaluate" in only:
        guarded(extras, "evaluate_tri512_M3_nv9", lambda: measure_evaluate(torch, C, res2["mesh"], Q2, 3, 2, 50))
    if "moving2d" in only:
        stored2 = {tag: res2[tag]["ms_per_step"] for tag in ("f64", "f32")}
        guarded(extras, "moving_tri512_M3_nv9", lambda: measure_moving(torch, C, m2, Q2, 3, "tri512 M3", 2, 10,
                                                                       stored2))
    if "weno" in only:
        guarded(extras, "weno_tri512_M3_nv9", lambda: measure_weno(torch, C, m2, Q2, 3, 2, 10,
                                                                   res2["f64"]["ms_per_step"], res2["n_e"]))
    if res2 is not None:
        res2.pop("mesh", None)

    # small mesh: launch-bound, reported as latency; every cell against the oracle
    if "tri64" in only:
        m1 = tri_mesh(64, 0.15, SEED1)
        Q1 = workload_fields(m1, "euler2d_sod", SEED1)
        r1 = measure(torch, C, m1, Q1, 2, 1.5, 200, 20, "tri64 M2", 2, keep_out=not args.no_oracle_error)
        extras["tri64_M2_nv4"] = {
            "workload": "2-D M=2, 8,192 jittered periodic triangles, n_e=9 (stencil factor 1.5), 4 Euler variables",
            "f64_latency_ms": r1["f64"]["latency_ms"], "f32_latency_ms": r1["f32"]["latency_ms"],
            "f64_value": r1["f64"]["value"], "f32_value": r1["f32"]["value"], "unit": "cells·vars/s"}
        if not args.no_oracle_error:
            t0 = time.perf_counter()
            parts = oracle_sample(m1, Q1, 2, 1.5, np.arange(m1.n_cells))
            errors["tri64_M2_nv4"] = oracle_error(parts, {t: r1[t]["out"] for t in ("f64", "f32")},
                                                  "every cell of the 2-D M=2 8,192-triangle mesh")
            errors["tri64_M2_nv4"]["oracle_s"] = time.perf_counter() - t0
        del r1

    if "batch" in only:
        guarded(extras, "batch64_mixed", lambda: measure_batch(torch, C, 20))
        if "oracle_error" in extras["batch64_mixed"]:
            errors["batch64_mixed"] = extras["batch64_mixed"]["oracle_error"]
    if "serving" in only and args.serve_seconds > 0:
        if args.serve_full:
            guarded(extras, "serving_full", lambda: measure_serving_full(torch, C, args.serve_seconds))
        else:
            guarded(extras, "serving", lambda: measure_serving(torch, C, args.serve_seconds))

    cpu = None
    if res3 is not None and not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, parts3 = cpu_baseline(m3, Q3, 3, 0.0, args.cpu_seconds, args.cpu_all_cores_seconds)
        log(f"cpu: {cpu['value']:.3e} cells*vars/s on one thread"
            + (f", {cpu['all_cores']['value']:.3e} on {cpu['all_cores']['cores']} processes"
               if "value" in cpu.get("all_cores", {}) else ""))
        if not args.no_oracle_error:
            errors["kuhn64_M3_nv5"] = oracle_error(parts3, {t: res3[t]["out"] for t in ("f64", "f32")},
                                                   "the cells of the CPU baseline's sample (random order)")
    if res2 is not None and "out" in res2["f64"]:
        t0 = time.perf_counter()
        cells2 = np.random.default_rng(SEED + 2).choice(m2.n_cells, size=8192, replace=False)
        parts = oracle_sample(m2, Q2, 3, 0.0, cells2)
        errors["tri512_M3_nv9"] = oracle_error(parts, {t: res2[t]["out"] for t in ("f64", "f32")},
                                               "8,192 seeded random cells")
        errors["tri512_M3_nv9"]["oracle_s"] = time.perf_counter() - t0
    for k, e in errors.items():
        if "f64_max" in e:
            log(f"oracle error {k}: FP64 max {e['f64_max']:.2e}, FP32 max {e['f32_max']:.2e}, "
                f"p99.9 {e['f32_p999']:.2e} over {e['cells_compared']} cells")

    line = {"metric": METRIC, "value": None, "unit": "cells·vars/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic"}
    if res3 is not None:
        r64 = res3["f64"]
        line.update({
            "value": r64["value"], "ms_per_step": r64["ms_per_step"],
            "config": {"workload": "CWENO 3-D M=3 (20 basis functions), 1,572,864 jittered periodic Kuhn "
                                   "tetrahedra (64^3 cubes x 6), n_e=60, 4 cone sectors, 5 Euler variables",
                       "cells": m3.n_cells, "n_vars": Q3.shape[0], "degree": 3, "dim": 3, "n_e": res3["n_e"],
                       "lambda0": 0.95, "eps": 1e-14, "r": 4, "seed": SEED3},
            "roofline": r64["roofline"],
            "latency_ms": r64["latency_ms"],
            "cache_flushed": {"f64_ms": r64["flushed_ms"], "f64_frac": r64["flushed_frac"],
                              "f32_ms": res3["f32"]["flushed_ms"], "f32_frac": res3["f32"]["flushed_frac"],
                              "note": "median single launch after a read-only pass over 1 GiB; value and "
                                      "roofline are back-to-back launches"},
            "kernel_variant": {"f64": r64["variant"], "f32": res3["f32"]["variant"]},
            "fp32": {"value": res3["f32"]["value"], "ms_per_step": res3["f32"]["ms_per_step"],
                     "latency_ms": res3["f32"]["latency_ms"], "roofline": res3["f32"]["roofline"],
                     "dtype": "f32", "error_vs_oracle": errors.get("kuhn64_M3_nv5")},
            "precompute_s": res3["precompute_s"],
            "precompute_device_operators_s": res3.get("precompute_device_operators_s")})
    line.update({"cpu_baseline": cpu, "oracle_error": errors, "extras": extras,
                 "kernel_source_sha": kernel_source_hash(),
                 "moving_kernel_source_sha": kernel_source_hash(MOVING_SRCS)})
    print(json.dumps(line))


if __name__ == "__main__":
    main()
