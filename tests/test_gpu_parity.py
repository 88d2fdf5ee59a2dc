"""GPU parity: the HIP reconstruction (through the C ABI) against the oracle.

FP64 bar: data-scaled error <= 1e-12 (each coefficient difference divided by
the largest |Q| of the cell's central stencil), indicators to 1e-9 relative,
weights to 1e-9 absolute; coefficient 0 is a bitwise copy of the input.
"""
import sys

import numpy as np
import pytest

from gpu_common import data_scaled_error, run_library, torch_cuda
from oracle import CwenoOracle, Options
from synthetic import kuhn_tet_mesh, tri_mesh, workload_fields

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _lib():
    import paper_1612_09335_amd as C
    return C


def _check_f64(m, M, Q, factor=0.0, cells=None, **opts):
    torch = torch_cuda()
    C = _lib()
    lib_opts = {k: v for k, v in opts.items() if k in ("sector_rule", "r", "eps")}
    if "lambda0" in opts:
        lib_opts["lambda0"] = -1.0 if opts["lambda0"] == "paper" else opts["lambda0"]
    if opts.get("sigma0_from") == "popt":
        lib_opts["sigma0_popt"] = True
    if opts.get("linear_weights"):
        lib_opts["linear_weights"] = True
    print(f"[gpu parity] {m.name} M={M} nv={Q.shape[0]} cells={m.n_cells} opts={opts}", flush=True)
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, stencil_factor=factor, **lib_opts)
    res = run_library(torch, lm, Q, torch.float64)
    assert np.array_equal(res["coeffs"][:, 0, :].view(np.int64), Q.view(np.int64))
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M, stencil_factor=factor, **opts))
    idx = np.arange(m.n_cells) if cells is None else np.asarray(cells)
    ref = o.reconstruct(Q, cells=idx)
    st = lm.tables()["stencil"][idx]
    err = data_scaled_error(res["coeffs"][:, :, idx], ref["coeffs"], Q, st)
    print(f"[gpu parity]   data-scaled coefficient error {err:.3e}", flush=True)
    assert err <= TOL64
    sg, om = res["sigma"][:, :, idx], res["omega"][:, :, idx]
    scale2 = (np.abs(Q[:, st]).max(axis=2) ** 2)[:, None, :]
    assert np.all(np.abs(sg - ref["sigma"]) <= 1e-9 * np.abs(ref["sigma"]) + 1e-20 * scale2)
    assert np.abs(om - ref["omega"]).max() <= 1e-9
    return lm, res


def test_cfg1_full_mesh_f64():
    """2-D M=2, 64x64x2 jittered periodic triangles, n_e = 9, Euler + Sod circle."""
    m = tri_mesh(64, 0.15, 16120934)
    Q = workload_fields(m, "euler2d_sod", 16120934)
    _check_f64(m, 2, Q, factor=1.5)


@pytest.mark.parametrize("case", ["tri13_M3_nv7", "kuhn5_M2_nv3", "tri12_M4_nv2", "kuhn6_M1_nv5",
                                  "tri10_M3_bounded", "kuhn4_M2_bounded"])
def test_small_meshes_f64(case):
    rng = np.random.default_rng(abs(hash(case)) % 2**32)
    if case == "tri13_M3_nv7":
        m, M, nv = tri_mesh(13, 0.15, 1), 3, 7
    elif case == "kuhn5_M2_nv3":
        m, M, nv = kuhn_tet_mesh(5, 0.1, 2), 2, 3
    elif case == "tri12_M4_nv2":
        m, M, nv = tri_mesh(12, 0.15, 3), 4, 2
    elif case == "kuhn6_M1_nv5":
        m, M, nv = kuhn_tet_mesh(6, 0.1, 4), 1, 5
    elif case == "tri10_M3_bounded":
        m, M, nv = tri_mesh(10, 0.15, 5, periodic=False), 3, 3
    else:
        m, M, nv = kuhn_tet_mesh(4, 0.1, 6, periodic=False), 2, 4
    Q = rng.normal(size=(nv, m.n_cells)) + 4.0 * (rng.random((1, m.n_cells)) < 0.25)
    _check_f64(m, M, Q)


@pytest.mark.parametrize("case", ["kuhn7_M4_nv5", "kuhn5_M3_nv9", "tri12_M4_nv9"])
def test_two_pass_blocks_f64(case):
    """Variable blocks whose FP64 accumulators exceed one lane's budget: the
    halo kernel walks the stencil twice, half of P_opt's rows each time (3-D
    degree 4 with 5 variables, 3-D degree 3 with 9, 2-D degree 4 with 9);
    ragged last block; sampled cells against the oracle."""
    rng = np.random.default_rng(abs(hash(case)) % 2**32)
    if case == "kuhn7_M4_nv5":
        m, M, nv = kuhn_tet_mesh(7, 0.1, 51), 4, 5
    elif case == "kuhn5_M3_nv9":
        m, M, nv = kuhn_tet_mesh(5, 0.1, 52), 3, 9
    else:
        m, M, nv = tri_mesh(12, 0.15, 53), 4, 9
    Q = rng.normal(size=(nv, m.n_cells)) + 4.0 * (rng.random((1, m.n_cells)) < 0.25)
    cells = np.unique(np.concatenate([rng.choice(m.n_cells, min(m.n_cells, 48), replace=False),
                                      np.arange(max(0, m.n_cells - 8), m.n_cells)]))
    lm, _ = _check_f64(m, M, Q, cells=cells)
    assert lm.get_variant("f64", nv if nv < 9 else 9)[0] >= 0


@pytest.mark.parametrize("opt", [dict(sector_rule="face"), dict(lambda0="paper"), dict(sigma0_from="popt"),
                                 dict(linear_weights=True), dict(r=2, eps=1e-6), dict(lambda0=0.5)])
def test_options_f64(opt):
    m = tri_mesh(11, 0.15, 21)
    rng = np.random.default_rng(22)
    Q = rng.normal(size=(2, m.n_cells)) + 3.0 * (rng.random((1, m.n_cells)) < 0.3)
    _check_f64(m, 3, Q, **opt)


def test_deterministic_and_stream_ordered():
    torch = torch_cuda()
    C = _lib()
    m = tri_mesh(32, 0.15, 31)
    Q = workload_fields(m, "mhd2d", 31)
    lm = C.Mesh(m.vertices, m.cells, 3, periodic=m.box)
    a = run_library(torch, lm, Q, torch.float64)["coeffs"]
    b = run_library(torch, lm, Q, torch.float64)["coeffs"]
    assert np.array_equal(a.view(np.int64), b.view(np.int64))


@pytest.mark.parametrize("case", ["tri13_M3_nv9", "kuhn6_M3_nv5", "tri12_M2_nv4", "tri10_M4_nv5", "kuhn5_M2_nv9",
                                  "kuhn7_M4_nv5"])
def test_every_variant_bitwise_identical(case):
    """All kernel variants (lanes per cell, stencil chunk) give the same bits,
    and the default one matches the oracle."""
    torch = torch_cuda()
    C = _lib()
    if case == "tri13_M3_nv9":
        m, M, nv = tri_mesh(13, 0.15, 41), 3, 9
    elif case == "kuhn6_M3_nv5":
        m, M, nv = kuhn_tet_mesh(6, 0.1, 42), 3, 5
    elif case == "tri12_M2_nv4":
        m, M, nv = tri_mesh(12, 0.15, 43), 2, 4
    elif case == "tri10_M4_nv5":
        m, M, nv = tri_mesh(10, 0.15, 44), 4, 5
    elif case == "kuhn7_M4_nv5":
        m, M, nv = kuhn_tet_mesh(7, 0.1, 47), 4, 5
    else:
        m, M, nv = kuhn_tet_mesh(5, 0.1, 45), 2, 9
    rng = np.random.default_rng(46)
    Q = rng.normal(size=(nv, m.n_cells)) + 3.0 * (rng.random((1, m.n_cells)) < 0.3)
    print(f"[gpu variants] {case}", flush=True)
    for dt, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops=dt)
        base = run_library(torch, lm, Q, tdt)
        seen = 0
        for vb in range(1, 10):
            k0 = lm.get_variant(dt, vb)[0]
            if k0 < 0:
                continue
            for k in range(C.num_variants()):
                try:
                    lm.set_variant(dt, vb, k)
                except C.CwenoError:
                    continue
                res = run_library(torch, lm, Q, tdt)
                for key in ("coeffs", "sigma", "omega"):
                    assert np.array_equal(res[key], base[key]), (dt, vb, k, key)
                seen += 1
            lm.set_variant(dt, vb, k0)
        assert seen >= 6
        if dt == "f64":
            o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
            ref = o.reconstruct(Q, cells=range(0, m.n_cells, 7))
            idx = np.arange(0, m.n_cells, 7)
            err = data_scaled_error(base["coeffs"][:, :, idx], ref["coeffs"], Q, lm.tables()["stencil"][idx])
            assert err <= TOL64


def test_more_variables_than_one_block_and_argument_errors():
    """11 variables run as several variable blocks; overlapping or missing
    buffers are refused before any launch."""
    torch = torch_cuda()
    C = _lib()
    m = tri_mesh(12, 0.15, 51)
    rng = np.random.default_rng(52)
    Q = rng.normal(size=(11, m.n_cells)) + 2.0 * (rng.random((1, m.n_cells)) < 0.3)
    lm, res = _check_f64(m, 2, Q)
    q = torch.tensor(Q, dtype=torch.float64, device="cuda:0")
    out = torch.empty((11, lm.n_basis, lm.n_cells), dtype=torch.float64, device="cuda:0")
    lib = C.lib
    # coefficients overlapping the averages
    big = torch.empty(11 * lm.n_basis * lm.n_cells + 11 * lm.n_cells, dtype=torch.float64, device="cuda:0")
    st = lib.cweno_reconstruct(lm._h, 11, C.F64, big.data_ptr(), big.data_ptr() + 8 * 5, None, None, None)
    assert st == -1 and b"overlap" in lib.cweno_last_error()
    # missing buffers, zero variables, wrong precision for the operators held
    assert lib.cweno_reconstruct(lm._h, 11, C.F64, None, out.data_ptr(), None, None, None) == -1
    assert lib.cweno_reconstruct(lm._h, 0, C.F64, q.data_ptr(), out.data_ptr(), None, None, None) == -1
    assert lib.cweno_reconstruct(lm._h, 11, C.F32, q.data_ptr(), out.data_ptr(), None, None, None) == -1



@pytest.mark.parametrize("d,M", [(2, 3), (3, 2)])
def test_renumbering_permutes_results(d, M):
    """Renumbering cells and vertices (each cell's own vertex order kept)
    permutes the tables and the coefficients and changes nothing else."""
    torch = torch_cuda()
    C = _lib()
    m = tri_mesh(14, 0.15, 61) if d == 2 else kuhn_tet_mesh(6, 0.1, 62)
    rng = np.random.default_rng(63)
    pc = rng.permutation(m.n_cells)                # new cell k is old cell pc[k]
    pv = rng.permutation(m.n_vertices)             # new vertex k is old vertex pv[k]
    inv_v = np.empty_like(pv)
    inv_v[pv] = np.arange(len(pv))
    V2 = m.vertices[pv]
    C2 = inv_v[m.cells[pc]].astype(np.int32)
    Q = rng.normal(size=(4, m.n_cells)) + 3.0 * (rng.random((1, m.n_cells)) < 0.3)
    a = C.Mesh(m.vertices, m.cells, M, periodic=m.box)
    b = C.Mesh(V2, C2, M, periodic=m.box)
    ta, tb = a.tables(), b.tables()
    assert np.array_equal(pc[tb["stencil"]], ta["stencil"][pc])
    sb = tb["sectors"]
    mapped = np.where(sb >= 0, pc[np.maximum(sb, 0)], -1)
    assert np.array_equal(mapped, ta["sectors"][pc])
    ra = run_library(torch, a, Q, torch.float64)
    rb = run_library(torch, b, Q[:, pc], torch.float64)
    err = data_scaled_error(rb["coeffs"], ra["coeffs"][:, :, pc], Q[:, pc], tb["stencil"])
    print(f"[gpu parity] renumbered d={d} M={M}: {err:.2e}", flush=True)
    assert err <= 1e-13
