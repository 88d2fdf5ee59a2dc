"""Pins of the oracle's classical unstructured WENO reconstruction (the
scheme the paper compares CWENO with, Sec. 4).

* Stencils: 1 + 2(d+1) of them, n_e distinct cells each, the cell first;
  every forward-sector cell has a barycentre with all barycentric coordinates
  but the s-th positive, every reverse-sector cell all but the s-th negative
  (re-derived here by solving the barycentric system directly).
* Every stencil's polynomial is of degree M and reproduces degree-M data, so
  the nonlinear blend reproduces any polynomial of degree <= M exactly from
  its exact averages, whatever the weights.
* Conservation: the blend's cell average is the input average.
* Across a jump the blend stays within the data range far better than the
  central polynomial alone.
"""
import numpy as np
import pytest

from oracle import CwenoOracle, Options, WenoOracle, evaluate_polynomial
from synthetic import cell_averages, kuhn_tet_mesh, polynomial_field, random_polynomial, tri_mesh


def _bary(o, i, j):
    X = np.array(o.cw.geo.cell_vertices(i))
    p = np.array(o.cw.geo.centroid(i)) + np.array(o.cw.geo.offset(i, j))
    d = X.shape[1]
    A = np.vstack([X.T, np.ones(d + 1)])
    return np.linalg.solve(A, np.append(p, 1.0))


@pytest.mark.parametrize("d,M,n", [(2, 2, 16), (2, 3, 24), (3, 2, 16)])
def test_stencils_sizes_and_cones(d, M, n):
    m = tri_mesh(n, 0.15, 701) if d == 2 else kuhn_tet_mesh(n, 0.1, 702)
    o = WenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    rng = np.random.default_rng(703)
    for i in rng.choice(m.n_cells, 6, replace=False):
        st = o.stencils(int(i))
        assert len(st) == 1 + 2 * (d + 1)
        for j, S in enumerate(st):
            assert S is not None and len(S) == o.n_e and S[0] == i and len(set(S)) == o.n_e
            if j == 0:
                continue
            s = (j - 1) % (d + 1)
            sign = 1.0 if j <= d + 1 else -1.0
            for c in S[1:]:
                b = _bary(o, int(i), c)
                assert all(sign * b[k] > 0 for k in range(d + 1) if k != s), (i, j, c, b)


@pytest.mark.parametrize("d,M,n", [(2, 2, 14), (2, 3, 20), (3, 2, 12)])
def test_blend_reproduces_polynomials(d, M, n):
    m = tri_mesh(n, 0.15, 710 + M, periodic=False) if d == 2 else kuhn_tet_mesh(n, 0.1, 711, periodic=False)
    fn = polynomial_field(random_polynomial(d, M, 2, seed=712 + M))
    Q = cell_averages(m, fn, degree=max(M, 5) if d == 2 else M + 1)
    o = WenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    ref = np.random.default_rng(713).dirichlet(np.ones(d + 1), size=5)[:, 1:]
    centre = np.array([0.5] * d)
    cents = m.vertices[m.cells].mean(axis=1)
    inner = np.argsort(np.linalg.norm(cents - centre, axis=1))[:4]
    for i in inner:
        r = o.reconstruct_cell(int(i), Q)
        assert r["alive"].all()
        X = np.array(o.cw.geo.cell_vertices(int(i)))
        phys = (X[0] + ref @ (X[1:] - X[0])).T
        got = evaluate_polynomial(M, d, r["coeffs"], ref)
        want = fn(phys)
        assert np.abs(got - want).max() <= 1e-10 * max(1.0, np.abs(want).max())


def test_conservation_and_jump():
    m = tri_mesh(24, 0.15, 720)
    o = WenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    cw = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    c = m.vertices[m.cells].mean(axis=1)
    Q = np.where(c[:, 0] < 0.5, 1.0, 0.1)[None, :] + 0.0 * c[:, 1][None, :]
    from oracle.quadrature import collapsed_rule
    pts, w = collapsed_rule(2, 3)
    near = [i for i in range(m.n_cells) if abs(c[i, 0] - 0.5) < 0.06][:12]
    worst_weno = worst_popt = 0.0
    for i in near:
        r = o.reconstruct_cell(i, Q)
        avg = evaluate_polynomial(3, 2, r["coeffs"], pts) @ w / w.sum()
        np.testing.assert_allclose(avg, Q[:, i], rtol=1e-13, atol=1e-13)
        vals = evaluate_polynomial(3, 2, r["coeffs"], pts)
        worst_weno = max(worst_weno, max(vals.max() - 1.0, 0.1 - vals.min()))
        popt = cw.reconstruct_cell(i, Q)["popt"]
        pv = evaluate_polynomial(3, 2, popt, pts)
        worst_popt = max(worst_popt, max(pv.max() - 1.0, 0.1 - pv.min()))
    assert worst_weno < 0.1 * worst_popt
