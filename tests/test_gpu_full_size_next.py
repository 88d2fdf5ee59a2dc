"""Parity at the benchmark's full sizes for the moving-mesh form, the point
values and the classical WENO scheme, in the configurations bench.py times.

* Moving mesh: the 2-D workload (524,288 triangles, M=3, 9 variables) and the
  3-D one (1,572,864 tetrahedra, M=3, 5 variables) with the benchmark's
  vertex motion; sampled cells against the oracle with the same fixed
  stencils (FP64 to 1e-12, FP32 to 2e-6 of the data scale); every cell
  finite with a bitwise coefficient 0; no fault reported.
* Point values: the benchmark reconstruction at the 12 face Gauss points;
  every cell against the oracle's evaluation of the same coefficients.
* Classical WENO: the 2-D workload; sampled cells against the oracle's WENO.
"""
import dataclasses

import numpy as np
import pytest

from gpu_common import data_scaled_error, torch_cuda
from oracle import CwenoOracle, Options, WenoOracle, evaluate_polynomial
from synthetic import kuhn_tet_mesh, moved_vertices, tri_mesh, workload_fields

pytestmark = pytest.mark.gpu

SEED2, SEED3 = 16120935, 16120936


def _moving_full(m, Q, M, n_sample, seed):
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops="none", moving=True)
    V = moved_vertices(m, 0.2, 0.1)                       # the benchmark's motion
    t = lm.tables()
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([rng.choice(m.n_cells, n_sample, replace=False), [0, m.n_cells - 1]]))
    o = CwenoOracle(V, m.cells, m.box, Options(degree=M), stencils=(t["stencil"], t["sectors"]))
    ref = o.reconstruct(Q, cells=idx)["coeffs"]
    vt = torch.tensor(V, device="cuda:0")
    for tdt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-6)):
        q = torch.tensor(Q, dtype=tdt, device="cuda:0")
        fault = torch.zeros(1, dtype=torch.int32, device="cuda:0")
        out = lm.reconstruct_moving(vt, q, fault=fault)
        torch.cuda.synchronize()
        assert int(fault.item()) == 0
        c = out.cpu().numpy().astype(np.float64)
        assert np.isfinite(c).all()
        assert np.array_equal(c[:, 0, :], Q.astype(np.float64 if tdt == torch.float64 else np.float32))
        err = data_scaled_error(c[:, :, idx], ref, Q, t["stencil"][idx])
        print(f"[gpu full next] moving {m.name} {tdt}: sampled error {err:.3e} over {len(idx)} cells", flush=True)
        assert err <= tol
        del q, out


@pytest.mark.timeout(900)
def test_moving_full_size_tri512():
    m = tri_mesh(512, 0.15, SEED2)
    _moving_full(m, workload_fields(m, "mhd2d", SEED2), 3, 200, 21)


@pytest.mark.timeout(900)
def test_moving_full_size_kuhn64():
    m = kuhn_tet_mesh(64, 0.1, SEED3)
    _moving_full(m, workload_fields(m, "euler3d_blast", SEED3), 3, 60, 22)


@pytest.mark.timeout(900)
def test_point_values_full_size_tri512():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = tri_mesh(512, 0.15, SEED2)
    Q = workload_fields(m, "mhd2d", SEED2)
    lm = C.Mesh(m.vertices, m.cells, 3, periodic=m.box, ops="both")
    g, _ = np.polynomial.legendre.leggauss(4)
    tt = 0.5 * (g + 1.0)
    verts = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    P = np.vstack([np.outer(1 - tt, verts[a]) + np.outer(tt, verts[b]) for a in range(3) for b in range(a + 1, 3)])
    pts = C.Points(2, 3, P)
    for tdt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-6)):
        co = lm.reconstruct(torch.tensor(Q, dtype=tdt, device="cuda:0"))
        vals = lm.evaluate(pts, co).cpu().numpy().astype(np.float64)
        c = co.cpu().numpy().astype(np.float64)
        for v in range(Q.shape[0]):
            want = evaluate_polynomial(3, 2, c[v].T, P).T           # [q, n]
            scale = np.abs(c[v]).sum(axis=0)[None, :]
            err = (np.abs(vals[v] - want) / np.maximum(scale, 1e-300)).max()
            assert err <= tol, (tdt, v, err)
        print(f"[gpu full next] point values {tdt}: every cell within {tol}", flush=True)


@pytest.mark.timeout(900)
def test_weno_full_size_tri512():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = tri_mesh(512, 0.15, SEED2)
    Q = workload_fields(m, "mhd2d", SEED2)
    lm = C.Mesh(m.vertices, m.cells, 3, periodic=m.box, weno=True)
    out = lm.reconstruct(torch.tensor(Q, device="cuda:0")).cpu().numpy()
    assert np.isfinite(out).all()
    assert np.array_equal(out[:, 0, :].view(np.int64), Q.view(np.int64))
    rng = np.random.default_rng(23)
    idx = np.unique(np.concatenate([rng.choice(m.n_cells, 40, replace=False), [0, m.n_cells - 1]]))
    o = WenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    ref = o.reconstruct(Q, cells=idx)["coeffs"]
    st = lm.weno_tables()[idx]
    scale = np.array([[np.abs(Q[v, s[s >= 0]]).max() for s in st.reshape(len(idx), -1)] for v in range(Q.shape[0])])
    err = (np.abs(out[:, :, idx] - ref) / scale[:, None, :]).max()
    print(f"[gpu full next] weno tri512: sampled error {err:.3e} over {len(idx)} cells", flush=True)
    assert err <= 1e-12
