"""Exact-rational brute force of the whole CWENO pipeline on tiny meshes.

Independent of the oracle's arithmetic: polynomials are kept in the monomial
basis of cell i's reference coordinates, stencil averages are integrated
exactly over each (dyadic-rational) simplex through barycentric monomial
integrals, P_opt comes from the KKT system of the equality-constrained least
squares problem (Sec. 2.1, eq. CWENO:Popt) solved by exact Gauss-Jordan
elimination, the sectorial P1 systems (eq. CWENO:Ps) likewise, and the
indicators sum_alpha int (d^alpha P)^2, the weights (eps = 1e-14 as an exact
rational, r = 4) and the blend are all exact.  Only the stencil tables are
taken from the oracle (they are pinned separately).  The comparison uses
basis-free quantities: point values, sigma and omega.  The exact arithmetic
lives in ``exact_rational.py``; dropped sectors, the face sector rule, sigma_0
of P_opt and the classical WENO weights have their own exact pins in
``test_oracle_options_exact.py``.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from exact_rational import exact_cweno, point_values
from oracle import CwenoOracle, Options, evaluate_polynomial
from synthetic import kuhn_tet_mesh, tri_mesh


@pytest.mark.parametrize("case", ["tri_M2", "tri_M3", "tet_M2"])
def test_pipeline_matches_exact_rational(case):
    if case.startswith("tri"):
        m = tri_mesh(8, 0.15, 21, periodic=False, dyadic=16)
        M = int(case[-1])
        cells = [2 * (8 * 3 + 3), 2 * (8 * 4 + 4) + 1]
    else:
        m = kuhn_tet_mesh(4, 0.1, 22, periodic=False, dyadic=16)
        M = 2
        cells = [6 * (16 * 1 + 4 * 2 + 1) + 2]
    rng = np.random.default_rng(5)
    # dyadic data with a jump so the weights are far from linear
    base = rng.integers(-64, 64, size=m.n_cells) / 16.0
    c = m.vertices[m.cells.astype(np.int64)].mean(axis=1)
    Q = np.stack([base, base + 8.0 * (c[:, 0] > 0.45), np.full(m.n_cells, 0.75)])
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    lam = [Fr(95, 100)] + [Fr(5, 100 * (m.dim + 1))] * (m.dim + 1)
    ref_pts = np.array([[0.0] * m.dim, [0.25] * m.dim, [0.5] + [0.125] * (m.dim - 1), [0.1] * m.dim])
    for i in cells:
        r = o.reconstruct_cell(i, Q)
        assert r["alive"].all()
        for v in range(Q.shape[0]):
            ex = exact_cweno(o, i, Q[v].tolist(), lam)
            assert all(ex["alive"])
            exact_vals = point_values(ex["cell"], ex["w"], ref_pts)
            got = evaluate_polynomial(M, m.dim, r["coeffs"][v], ref_pts)
            scale = max(1.0, np.abs(Q[v, o.stencils(i)[0]]).max())
            np.testing.assert_allclose(got, exact_vals, rtol=0, atol=1e-12 * scale)
            np.testing.assert_allclose(r["sigma"][v], [float(s) for s in ex["sigma"]], rtol=1e-10,
                                       atol=1e-22 * scale ** 2)
            np.testing.assert_allclose(r["omega"][v], [float(x) for x in ex["omega"]], rtol=0, atol=1e-12)
