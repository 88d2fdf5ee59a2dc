"""Pins of the oracle on moving meshes (fixed stencils, moved vertices).

On a moving mesh the connectivity and the stencils stay those of the mesh as
created, while every reconstruction matrix is rebuilt from the moved vertex
positions (Sec. 2.1 on ALE meshes).  The oracle takes the fixed stencils as
tables; these pins check that

* fixed tables equal to the selected ones change nothing (bit for bit);
* on a moved mesh, P_opt still reproduces every polynomial of degree <= M
  from its exact averages over the *moved* cells (whatever the stencil, the
  least-squares residual of such data is zero), so the moved frames, the
  moved averages and the moved quadrature all enter correctly;
* the result keeps the cell average (conservation) on the moved mesh;
* moving a vertex by a whole period of a periodic box changes nothing (the
  minimum image is taken on the moved positions).
"""
import dataclasses

import numpy as np
import pytest

from oracle import CwenoOracle, Options, evaluate_polynomial
from synthetic import (cell_averages, kuhn_tet_mesh, moved_vertices, polynomial_field, random_polynomial,
                       tri_mesh)


def _mesh(d, n, seed, periodic=True):
    return tri_mesh(n, 0.15, seed, periodic) if d == 2 else kuhn_tet_mesh(n, 0.1, seed, periodic)


def _fixed(o):
    t = o.tables()
    return t["stencil"], t["sectors"]


def _ref_points(d, k=6, seed=1):
    return np.random.default_rng(seed).dirichlet(np.ones(d + 1), size=k)[:, 1:]


def _phys(o, i, ref):
    X = np.array(o.geo.cell_vertices(i))
    return (X[0] + ref @ (X[1:] - X[0])).T


def test_fixed_tables_equal_to_selected_change_nothing():
    m = _mesh(2, 7, 901)
    Q = np.random.default_rng(902).normal(size=(3, m.n_cells))
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=2))
    f = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=2), stencils=_fixed(o))
    cells = list(range(0, m.n_cells, 5))
    a, b = o.reconstruct(Q, cells=cells), f.reconstruct(Q, cells=cells)
    for k in ("coeffs", "sigma", "omega"):
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("d,M,n", [(2, 2, 8), (2, 3, 8), (3, 2, 4), (3, 3, 5)])
def test_moved_mesh_popt_reproduces_polynomials(d, M, n):
    m = _mesh(d, n, 910 + M, periodic=False)
    base = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    V = moved_vertices(m, 0.3, 0.1)
    mm = dataclasses.replace(m, vertices=V)
    poly = random_polynomial(d, M, 2, seed=920 + M)
    fn = polynomial_field(poly)
    Q = cell_averages(mm, fn, degree=max(M, 5) if d == 2 else M + 1)
    o = CwenoOracle(V, m.cells, m.box, Options(degree=M), stencils=_fixed(base))
    ref = _ref_points(d)
    rng = np.random.default_rng(930)
    for i in rng.choice(m.n_cells, 6, replace=False):
        r = o.reconstruct_cell(int(i), Q)
        got = evaluate_polynomial(M, d, r["popt"], ref)
        want = fn(_phys(o, int(i), ref))
        assert np.abs(got - want).max() <= 1e-11 * max(1.0, np.abs(want).max())
    # the moved frame differs from the original one: the original operators do not reproduce the data
    i = int(rng.choice(m.n_cells))
    wrong = base.reconstruct_cell(i, Q)["popt"]
    want = fn(_phys(o, i, ref))
    assert np.abs(evaluate_polynomial(M, d, wrong, ref) - want).max() > 1e-6


@pytest.mark.parametrize("d,M", [(2, 3), (3, 2)])
def test_moved_mesh_conservation(d, M):
    m = _mesh(d, 8 if d == 2 else 4, 940)
    base = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    V = moved_vertices(m, 0.3, 0.37)
    rng = np.random.default_rng(941)
    Q = rng.normal(size=(2, m.n_cells)) + 5.0 * (rng.random(m.n_cells) < 0.3)
    o = CwenoOracle(V, m.cells, m.box, Options(degree=M), stencils=_fixed(base))
    from oracle.quadrature import collapsed_rule
    pts, w = collapsed_rule(d, M)
    for i in range(0, m.n_cells, max(1, m.n_cells // 8)):
        r = o.reconstruct_cell(i, Q)
        avg = evaluate_polynomial(M, d, r["coeffs"], pts) @ w / w.sum()
        np.testing.assert_allclose(avg, Q[:, i], rtol=1e-13, atol=1e-13)


def test_whole_period_vertex_shift_changes_nothing():
    m = _mesh(2, 8, 950)
    base = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    V = moved_vertices(m, 0.25, 0.2)
    V2 = V.copy()
    rng = np.random.default_rng(951)
    pick = rng.choice(m.n_vertices, m.n_vertices // 3, replace=False)
    V2[pick, 0] += 1.0
    V2[pick[::2], 1] -= 1.0
    Q = rng.normal(size=(2, m.n_cells))
    a = CwenoOracle(V, m.cells, m.box, Options(degree=3), stencils=_fixed(base))
    b = CwenoOracle(V2, m.cells, m.box, Options(degree=3), stencils=_fixed(base))
    cells = list(range(0, m.n_cells, 4))
    np.testing.assert_allclose(b.reconstruct(Q, cells=cells)["coeffs"], a.reconstruct(Q, cells=cells)["coeffs"],
                               rtol=0, atol=1e-11)
