"""GPU tests of the point values of the reconstruction (cweno_evaluate).

* The values at reference points (random interior points, the vertices, edge
  midpoints, Gauss points on the faces) equal the oracle's evaluation of the
  same coefficients: to 1e-13 of the coefficients' scale in FP64 and 1e-6 in
  FP32.
* End to end, against analytic values: with the linear weights forced
  (w = P_opt), the reconstruction of the exact averages of a degree-M
  polynomial, evaluated at reference points, equals that polynomial at the
  corresponding physical points of every cell.
"""
import numpy as np
import pytest

from gpu_common import torch_cuda
from oracle import evaluate_polynomial
from synthetic import cell_averages, kuhn_tet_mesh, polynomial_field, random_polynomial, tri_mesh

pytestmark = pytest.mark.gpu


def _ref_points(d, seed):
    rng = np.random.default_rng(seed)
    pts = [rng.dirichlet(np.ones(d + 1), size=7)[:, 1:]]
    verts = np.vstack([np.zeros(d), np.eye(d)])
    pts.append(verts)
    pts.append(np.array([(verts[a] + verts[b]) / 2 for a in range(d + 1) for b in range(a + 1, d + 1)]))
    g = 0.5 + 0.5 * np.array([-1, 1]) / np.sqrt(3.0)          # 2-point Gauss-Legendre on [0, 1]
    for a in range(d + 1):                                     # on each edge
        for b in range(a + 1, d + 1):
            pts.append(np.outer(1 - g, verts[a]) + np.outer(g, verts[b]))
    return np.vstack(pts)


CASES = [("tri11_M2", lambda: tri_mesh(11, 0.15, 601), 2, 4), ("tri12_M3", lambda: tri_mesh(12, 0.15, 602), 3, 9),
         ("tri10_M4", lambda: tri_mesh(10, 0.15, 603), 4, 3), ("kuhn4_M2", lambda: kuhn_tet_mesh(4, 0.1, 604), 2, 5),
         ("kuhn5_M3", lambda: kuhn_tet_mesh(5, 0.1, 605), 3, 5), ("kuhn4_M1", lambda: kuhn_tet_mesh(4, 0.1, 606), 1, 2)]


@pytest.mark.parametrize("name,mk,M,nv", CASES)
def test_point_values_match_oracle_evaluation(name, mk, M, nv):
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = mk()
    d = m.dim
    print(f"[gpu evaluate] {name}: {m.n_cells} cells", flush=True)
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops="both")
    P = _ref_points(d, 610 + M)
    pts = C.Points(d, M, P)
    assert np.abs(pts.basis() - np.asarray([evaluate_polynomial(M, d, np.eye(lm.n_basis), P[k:k + 1])[:, 0]
                                            for k in range(len(P))])).max() <= 1e-13
    rng = np.random.default_rng(611)
    Q = rng.normal(size=(nv, m.n_cells)) + 3.0 * (rng.random((1, m.n_cells)) < 0.3)
    for tdt, tol in ((torch.float64, 1e-13), (torch.float32, 1e-6)):
        q = torch.tensor(Q, dtype=tdt, device="cuda:0")
        co = lm.reconstruct(q)
        vals = torch.full((nv, len(P), m.n_cells), float("nan"), dtype=tdt, device="cuda:0")
        lm.evaluate(pts, co, out=vals)
        torch.cuda.synchronize()
        c = co.cpu().numpy().astype(np.float64)                       # [nv, nb, n]
        want = evaluate_polynomial(M, d, c.transpose(0, 2, 1), P)      # [nv, n, q]
        got = vals.cpu().numpy().astype(np.float64).transpose(0, 2, 1)
        scale = np.abs(c).sum(axis=1)[:, :, None]                      # sum_l |c_l| per cell and variable
        err = (np.abs(got - want) / np.maximum(scale, 1e-300)).max()
        print(f"[gpu evaluate]   {tdt}: max error / sum|c| = {err:.2e}", flush=True)
        assert err <= tol


@pytest.mark.parametrize("d,M", [(2, 3), (3, 2)])
def test_polynomial_reproduced_at_physical_points(d, M):
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = tri_mesh(10, 0.15, 620, periodic=False) if d == 2 else kuhn_tet_mesh(4, 0.1, 621, periodic=False)
    fn = polynomial_field(random_polynomial(d, M, 2, seed=622))
    Q = cell_averages(m, fn, degree=max(M, 5) if d == 2 else M + 1)
    lm = C.Mesh(m.vertices, m.cells, M, linear_weights=True)
    P = _ref_points(d, 623)
    pts = C.Points(d, M, P)
    q = torch.tensor(Q, device="cuda:0")
    vals = lm.evaluate(pts, lm.reconstruct(q)).cpu().numpy()           # [2, q, n]
    X = m.vertices[m.cells]                                            # [n, d+1, d]
    phys = X[:, 0, None, :] + np.einsum("qa,nab->nqb", P, X[:, 1:, :] - X[:, :1, :])   # [n, q, d]
    exact = fn(phys.reshape(-1, d).T).reshape(2, m.n_cells, len(P)).transpose(0, 2, 1)
    err = np.abs(vals - exact).max() / max(1.0, np.abs(exact).max())
    print(f"[gpu evaluate] d={d} M={M}: polynomial reproduction error {err:.2e}", flush=True)
    assert err <= 1e-10


def test_evaluate_arguments():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = tri_mesh(8, 0.15, 630)
    lm = C.Mesh(m.vertices, m.cells, 2, periodic=m.box)
    co = lm.reconstruct(torch.zeros((2, lm.n_cells), dtype=torch.float64, device="cuda:0"))
    with pytest.raises(C.CwenoError):
        lm.evaluate(C.Points(2, 3, [[0.2, 0.2]]), co)                 # point set of another degree
    with pytest.raises(C.CwenoError):
        C.Points(2, 2, np.zeros((0, 2)))
    pts = C.Points(2, 2, [[0.25, 0.25], [0.5, 0.0]])
    buf = torch.zeros(2 * lm.n_basis * lm.n_cells + 4 * lm.n_cells, dtype=torch.float64, device="cuda:0")
    st = C.lib.cweno_evaluate(lm._h, pts._h, 2, C.F64, buf.data_ptr(), buf.data_ptr() + 8, None)
    assert st == -1 and b"overlap" in C.lib.cweno_last_error()
    v = lm.evaluate(pts, co)
    torch.cuda.synchronize()
    assert torch.count_nonzero(v).item() == 0


FUSED = [("tri12_M3_nv9", lambda: tri_mesh(12, 0.15, 640), 3, 9), ("tri11_M2_nv7", lambda: tri_mesh(11, 0.15, 641), 2, 7),
         ("tri10_M4_nv3", lambda: tri_mesh(10, 0.15, 642), 4, 3), ("kuhn5_M3_nv5", lambda: kuhn_tet_mesh(5, 0.1, 643), 3, 5),
         ("kuhn4_M2_nv11", lambda: kuhn_tet_mesh(4, 0.1, 644), 2, 11),
         ("tri12_M3_bounded_nv4", lambda: tri_mesh(12, 0.15, 645, periodic=False), 3, 4)]


@pytest.mark.parametrize("name,mk,M,nv", FUSED)
def test_fused_point_values_equal_reconstruct_then_evaluate(name, mk, M, nv):
    """cweno_reconstruct_points gives the bits of cweno_reconstruct followed by
    cweno_evaluate (same blend, same sums in the same order)."""
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = mk()
    d = m.dim
    print(f"[gpu evaluate] fused {name}: {m.n_cells} cells", flush=True)
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops="both")
    pts = C.Points(d, M, _ref_points(d, 650 + M))
    rng = np.random.default_rng(651)
    Q = rng.normal(size=(nv, m.n_cells)) + 3.0 * (rng.random((1, m.n_cells)) < 0.3)
    for tdt in (torch.float64, torch.float32):
        q = torch.tensor(Q, dtype=tdt, device="cuda:0")
        two = lm.evaluate(pts, lm.reconstruct(q))
        fused = torch.full_like(two, float("nan"))
        lm.reconstruct_points(pts, q, out=fused)
        torch.cuda.synchronize()
        assert torch.equal(fused, two), (name, tdt)


def test_fused_point_values_refusals():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = tri_mesh(16, 0.15, 660)
    pts = C.Points(2, 2, [[0.2, 0.3]])
    w = C.Mesh(m.vertices, m.cells, 2, periodic=m.box, weno=True)
    q = torch.zeros((2, w.n_cells), dtype=torch.float64, device="cuda:0")
    with pytest.raises(C.CwenoError):
        w.reconstruct_points(pts, q)                            # WENO mesh
    f64 = C.Mesh(m.vertices, m.cells, 2, periodic=m.box, ops="f64")
    with pytest.raises(C.CwenoError):
        f64.reconstruct_points(pts, q.float())                  # no FP32 operators
    with pytest.raises(C.CwenoError):
        f64.reconstruct_points(C.Points(2, 3, [[0.2, 0.3]]), q)  # point set of another degree
