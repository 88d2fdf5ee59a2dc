"""Property pins of the oracle's reconstruction (Sec. 2.1).

* P_opt reproduces every polynomial of degree <= M from its exact cell
  averages on arbitrary (jittered) meshes: the least-squares residual is zero.
* Linear data: every sectorial P1 and P0 equal the data, all indicators are
  equal, so omega = lambda and w = data.  Constant data: sigma = 0, omega =
  lambda.
* With omega forced to lambda, w = P_opt, hence w reproduces degree <= M.
* Conservation: the reconstruction's cell average is the input average.
* Convergence: |P_opt - f| = O(h^(M+1)) on smooth data (nominal order M+1).
* omega -> lambda on smooth data as h -> 0.
* Across a jump the blend stays within the data range far better than
  P_opt (essentially non-oscillatory).
* Invariance under rotation + translation + scaling of the mesh, and under
  adding a constant to the data.
"""
import math

import numpy as np
import pytest

from oracle import CwenoOracle, Options, evaluate_polynomial, linear_weights
from synthetic import (cell_averages, kuhn_tet_mesh, polynomial_field, random_polynomial, tri_mesh)
from synthetic.meshes import SimplexMesh


def _mesh(d, n, seed, periodic=False):
    return tri_mesh(n, 0.15, seed, periodic) if d == 2 else kuhn_tet_mesh(n, 0.1, seed, periodic)


def _interior_cells(o, m, k, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in rng.permutation(m.n_cells):
        _, sec = o.stencils(int(i))
        if all(s is not None for s in sec):
            out.append(int(i))
        if len(out) == k:
            break
    return out


def _ref_points(d, k=6, seed=1):
    return np.random.default_rng(seed).dirichlet(np.ones(d + 1), size=k)[:, 1:]


def _phys(o, i, ref):
    X = np.array(o.geo.cell_vertices(i))
    return (X[0] + ref @ (X[1:] - X[0])).T


@pytest.mark.parametrize("d,M,n,k", [(2, 1, 6, 8), (2, 2, 8, 8), (2, 3, 8, 8), (2, 4, 10, 6),
                                     (3, 1, 3, 6), (3, 2, 4, 6), (3, 3, 5, 4)])
def test_popt_reproduces_polynomials(d, M, n, k):
    m = _mesh(d, n, 30 + M)
    poly = random_polynomial(d, M, 2, seed=40 + M)
    f = polynomial_field(poly)
    Q = cell_averages(m, f, degree=max(M, 5) if d == 2 else M + 1)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    ref = _ref_points(d)
    rng = np.random.default_rng(2)
    for i in rng.choice(m.n_cells, k, replace=False):
        r = o.reconstruct_cell(int(i), Q)
        got = evaluate_polynomial(M, d, r["popt"], ref)
        want = f(_phys(o, int(i), ref))
        assert np.abs(got - want).max() <= 1e-11 * max(1.0, np.abs(want).max())


@pytest.mark.parametrize("d,M", [(2, 3), (3, 2)])
def test_linear_data_gives_linear_weights(d, M):
    m = _mesh(d, 8 if d == 2 else 4, 51)
    f = polynomial_field(random_polynomial(d, 1, 2, seed=52))
    Q = cell_averages(m, f, degree=2)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    lam = linear_weights(d, 0.95)
    ref = _ref_points(d)
    for i in _interior_cells(o, m, 5):
        r = o.reconstruct_cell(i, Q)
        want = f(_phys(o, i, ref))
        for P in [r["popt"], r["p0"], r["coeffs"]] + [r["psec"][:, s] for s in range(d + 1)]:
            np.testing.assert_allclose(evaluate_polynomial(M, d, P, ref), want, atol=1e-11)
        np.testing.assert_allclose(r["omega"], np.tile(lam, (2, 1)), atol=1e-9)
        sig = r["sigma"]
        np.testing.assert_allclose(sig, np.repeat(sig[:, :1], d + 2, axis=1), rtol=1e-8)


def test_constant_data():
    m = tri_mesh(8, 0.15, 60, periodic=True)
    Q = np.full((2, m.n_cells), 3.25)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    r = o.reconstruct(Q, cells=range(0, m.n_cells, 7))
    assert np.abs(r["sigma"]).max() < 1e-24
    np.testing.assert_allclose(r["omega"], np.broadcast_to(linear_weights(2, 0.95)[None, :, None], r["omega"].shape), atol=1e-12)
    np.testing.assert_allclose(r["coeffs"][:, 0], 3.25, rtol=1e-15)
    assert np.abs(r["coeffs"][:, 1:]).max() < 1e-13


@pytest.mark.parametrize("d,M", [(2, 3), (3, 2)])
def test_linear_weight_mode_reproduces_degree_M(d, M):
    m = _mesh(d, 8 if d == 2 else 4, 70)
    f = polynomial_field(random_polynomial(d, M, 1, seed=71))
    Q = cell_averages(m, f, degree=max(M, 5) if d == 2 else M + 1)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M, linear_weights=True))
    ref = _ref_points(d)
    for i in _interior_cells(o, m, 4):
        r = o.reconstruct_cell(i, Q)
        want = f(_phys(o, i, ref))
        np.testing.assert_allclose(evaluate_polynomial(M, d, r["coeffs"], ref), want, atol=1e-11)


@pytest.mark.parametrize("d,M", [(2, 2), (2, 4), (3, 3)])
def test_conservation(d, M):
    m = _mesh(d, 8 if d == 2 else 6, 80, periodic=True)
    rng = np.random.default_rng(81)
    Q = rng.normal(size=(3, m.n_cells)) + 10.0 * (rng.random(m.n_cells) < 0.3)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    from oracle.quadrature import collapsed_rule
    pts, w = collapsed_rule(d, M)
    for i in range(0, m.n_cells, max(1, m.n_cells // 10)):
        r = o.reconstruct_cell(i, Q)
        # exact in exact arithmetic; the oracle's rounding is relative to the stencil's data scale
        scale = np.abs(Q[:, r["stencil"]]).max(axis=1)
        assert np.all(np.abs(r["coeffs"][:, 0] - Q[:, i]) <= 16 * np.finfo(float).eps * scale)
        avg = evaluate_polynomial(M, d, r["coeffs"], pts) @ w / w.sum()
        np.testing.assert_allclose(avg, Q[:, i], rtol=1e-14, atol=1e-14)


def _smooth(x):
    return np.stack([np.sin(2 * np.pi * x[0]) * np.cos(2 * np.pi * x[1])])


def _errors(d, M, n, paper_lambda=False, samples=150):
    """(max point error of w, of P_opt, median over cells of max_s |omega_s - lambda_s|)."""
    m = _mesh(d, n, 90, periodic=True)
    Q = cell_averages(m, _smooth, degree=9 if d == 2 else 7)
    o = CwenoOracle(m.vertices, m.cells, m.box,
                    Options(degree=M, lambda0="paper" if paper_lambda else 0.95))
    ref = _ref_points(d, 10, 3)
    ew = eo = 0.0
    dev = []
    for i in range(0, m.n_cells, max(1, m.n_cells // samples)):
        r = o.reconstruct_cell(i, Q)
        f = _smooth(_phys(o, i, ref))
        ew = max(ew, np.abs(evaluate_polynomial(M, d, r["coeffs"], ref) - f).max())
        eo = max(eo, np.abs(evaluate_polynomial(M, d, r["popt"], ref) - f).max())
        dev.append(np.abs(r["omega"] - o.lam[None, :]).max())
    return ew, eo, float(np.median(dev))


@pytest.mark.parametrize("M", [1, 2, 3])
def test_convergence_of_popt(M):
    _, e1, _ = _errors(2, M, 16)
    _, e2, _ = _errors(2, M, 32)
    rate = math.log2(e1 / e2)
    assert abs(rate - (M + 1)) < 0.5, rate


def test_weights_tend_to_linear_on_smooth_data():
    # eps = 1e-14 is absolute, so near critical points of the data all
    # indicators are tiny and omega departs from lambda; the typical cell
    # (median) approaches lambda at about O(h).
    _, _, d1 = _errors(2, 2, 32)
    _, _, d2 = _errors(2, 2, 64)
    assert d2 < 0.55 * d1
    # with the paper's lambda_0 = 1e5/(1e5+3) the blend is as accurate as P_opt
    ew, eo, _ = _errors(2, 2, 64, paper_lambda=True)
    assert ew <= 1.05 * eo


def test_no_overshoot_across_jump():
    """Cells near a unit jump but not cut by it: P_opt overshoots the stencil's
    data range at most of them, the blend at almost none."""
    m = tri_mesh(24, 0.15, 95, periodic=True)
    jump = lambda x: np.stack([np.where(x[0] < 0.5, 1.0, 0.0)])
    Q = cell_averages(m, jump, degree=5)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    ref = _ref_points(2, 12, 4)
    n = bad_w = bad_opt = 0
    for i in range(m.n_cells):
        c = np.array(o.geo.centroid(i))
        if min(abs(c[0] - 0.5), abs(c[0]), abs(c[0] - 1.0)) > 2.5 / 24 or 0.0 < Q[0, i] < 1.0:
            continue
        r = o.reconstruct_cell(i, Q)
        S = o.stencils(i)[0]
        lo, hi = Q[0, S].min(), Q[0, S].max()
        n += 1
        for P, which in ((r["coeffs"], "w"), (r["popt"], "o")):
            v = evaluate_polynomial(3, 2, P, ref)
            if max(v.max() - hi, lo - v.min()) > 1e-3:
                if which == "w":
                    bad_w += 1
                else:
                    bad_opt += 1
    assert n > 300
    assert bad_opt > 0.5 * n
    assert bad_w <= 0.01 * n


def test_similarity_and_shift_invariance():
    m = tri_mesh(8, 0.15, 99, periodic=False)
    rng = np.random.default_rng(100)
    Q = rng.normal(size=(2, m.n_cells))
    o1 = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    V2 = 3.0 * m.vertices @ R.T + np.array([5.0, -2.0])
    m2 = SimplexMesh(2, V2, m.cells, (0.0, 0.0), m.h * 3)
    o2 = CwenoOracle(m2.vertices, m2.cells, m2.box, Options(degree=3))
    o3 = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    for i in _interior_cells(o1, m, 6):
        r1 = o1.reconstruct_cell(i, Q)
        r2 = o2.reconstruct_cell(i, Q)
        assert r1["stencil"] == r2["stencil"] and r1["sectors"] == r2["sectors"]
        np.testing.assert_allclose(r2["coeffs"], r1["coeffs"], atol=1e-12)
        r3 = o3.reconstruct_cell(i, Q + 7.5)
        np.testing.assert_allclose(r3["coeffs"][:, 1:], r1["coeffs"][:, 1:], atol=1e-12)
        np.testing.assert_allclose(r3["omega"], r1["omega"], atol=1e-12)
