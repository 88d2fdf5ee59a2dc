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
basis-free quantities: point values, sigma and omega.
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import CwenoOracle, Options, evaluate_polynomial
from synthetic import kuhn_tet_mesh, tri_mesh


def _exps(d, M):
    out = []
    for n in range(M + 1):
        for e in itertools.product(range(n + 1), repeat=d):
            if sum(e) == n:
                out.append(e)
    return out


def _poly_mul(a, b):
    out = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, Fr(0)) + va * vb
    return out


def _simplex_avg_monomial(Y, e):
    """Exact average over the simplex with vertices Y of prod x_a^e_a.

    x_a = sum_k lam_k Y[k][a]; the average of prod lam_k^K_k over a simplex is
    d! prod K_k! / (|K| + d)!.
    """
    d = len(Y) - 1
    poly = {(0,) * (d + 1): Fr(1)}
    for a, p in enumerate(e):
        lin = {}
        for k in range(d + 1):
            key = tuple(1 if t == k else 0 for t in range(d + 1))
            lin[key] = Y[k][a]
        for _ in range(p):
            poly = _poly_mul(poly, lin)
    tot = Fr(0)
    for K, c in poly.items():
        tot += c * Fr(math.factorial(d) * math.prod(math.factorial(k) for k in K), math.factorial(sum(K) + d))
    return tot


def _solve(A, b):
    """Exact Gauss-Jordan with pivot search; A square list of lists."""
    n = len(A)
    M = [list(A[r]) + [b[r]] for r in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[r][n] for r in range(n)]


def _ref_integral(e):
    return Fr(math.prod(math.factorial(k) for k in e), math.factorial(sum(e) + len(e)))


def _sigma(coef, exps, d, M):
    """sum over distinct alpha, 1 <= |alpha| <= M, of int_{T_E} (d^alpha P)^2."""
    tot = Fr(0)
    for alpha in _exps(d, M)[1:]:
        der = {}
        for c, e in zip(coef, exps):
            if c == 0 or any(e[a] < alpha[a] for a in range(d)):
                continue
            f = c
            for a in range(d):
                for t in range(alpha[a]):
                    f *= e[a] - t
            ne = tuple(e[a] - alpha[a] for a in range(d))
            der[ne] = der.get(ne, Fr(0)) + f
        sq = _poly_mul(der, der)
        tot += sum((c * _ref_integral(k) for k, c in sq.items()), Fr(0))
    return tot


def _frac_vertices(o, i, j):
    return [[Fr(float(x)) for x in row] for row in o.geo.vertices_in_frame_of(i, j)]


def exact_cweno(o, i, Qcol, lam):
    """Exact reconstruction of one variable at cell i; returns (w, sigma, omega, exps)."""
    d, M = o.d, o.M
    exps = _exps(d, M)
    Xi = [[Fr(float(x)) for x in row] for row in o.geo.cell_vertices(i)]
    J = [[Xi[k + 1][a] - Xi[0][a] for k in range(d)] for a in range(d)]
    # inverse of J exactly (columns solved one by one)
    Jinv_cols = [_solve(J, [Fr(int(r == c)) for r in range(d)]) for c in range(d)]
    Jinv = [[Jinv_cols[c][r] for c in range(d)] for r in range(d)]

    def to_ref(x):
        y = [x[a] - Xi[0][a] for a in range(d)]
        return [sum((Jinv[r][a] * y[a] for a in range(d)), Fr(0)) for r in range(d)]

    def row_of(j):
        Y = [to_ref(v) for v in _frac_vertices(o, i, j)]
        return [_simplex_avg_monomial(Y, e) for e in exps]

    S0, sectors = o.stencils(i)
    A = [row_of(j) for j in S0]
    q = [Fr(Qcol[j]) for j in S0]
    nm = len(exps)
    # KKT: [2 A^T A  a0^T; a0 0] [p; mu] = [2 A^T q; q0]
    K = [[2 * sum((A[k][r] * A[k][c] for k in range(len(A))), Fr(0)) for c in range(nm)] + [A[0][r]]
         for r in range(nm)]
    K.append(A[0] + [Fr(0)])
    rhs = [2 * sum((A[k][r] * q[k] for k in range(len(A))), Fr(0)) for r in range(nm)] + [q[0]]
    popt = _solve(K, rhs)[:nm]

    lin = [exps.index(e) for e in exps if sum(e) <= 1]
    polys = []
    for sec in sectors:
        As = [[row_of(j)[t] for t in lin] for j in sec]
        ps = _solve(As, [Fr(Qcol[j]) for j in sec])
        full = [Fr(0)] * nm
        for t, v in zip(lin, ps):
            full[t] = v
        polys.append(full)
    p0 = [(popt[t] - sum((lam[s + 1] * polys[s][t] for s in range(d + 1)), Fr(0))) / lam[0] for t in range(nm)]
    allp = [p0] + polys
    sig = [_sigma(p, exps, d, M) for p in allp]
    eps = Fr(1, 10 ** 14)
    wt = [lam[s] / (sig[s] + eps) ** 4 for s in range(d + 2)]
    tot = sum(wt, Fr(0))
    om = [x / tot for x in wt]
    w = [sum((om[s] * allp[s][t] for s in range(d + 2)), Fr(0)) for t in range(nm)]
    return w, sig, om, exps


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
            w, sig, om, exps = exact_cweno(o, i, Q[v].tolist(), lam)
            exact_vals = [float(sum((w[t] * math.prod(Fr(p[a]) ** exps[t][a] for a in range(m.dim))
                                     for t in range(len(exps))), Fr(0))) for p in ref_pts]
            got = evaluate_polynomial(M, m.dim, r["coeffs"][v], ref_pts)
            scale = max(1.0, np.abs(Q[v, o.stencils(i)[0]]).max())
            np.testing.assert_allclose(got, exact_vals, rtol=0, atol=1e-12 * scale)
            np.testing.assert_allclose(r["sigma"][v], [float(s) for s in sig], rtol=1e-10, atol=1e-22 * scale ** 2)
            np.testing.assert_allclose(r["omega"][v], [float(x) for x in om], rtol=0, atol=1e-12)
