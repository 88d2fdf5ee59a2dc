"""Pins for the oracle's basis, oscillation matrix and quadrature.

Each check compares against something other than the oracle's own formula:
the paper's printed DOF totals, hand-derived closed forms, scipy's Jacobi
polynomials evaluated in collapsed coordinates, and sympy's symbolic
integration over the reference simplex.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp
from scipy.special import eval_jacobi

from oracle import basis as B
from oracle.quadrature import collapsed_rule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
xi, eta, zeta = sp.symbols("xi eta zeta")


def _to_sympy(poly, d):
    syms = (xi, eta, zeta)[:d]
    out = 0
    for e, c in poly.items():
        term = sp.Rational(c.numerator, c.denominator)
        for a in range(d):
            term *= syms[a] ** e[a]
        out += term
    return sp.expand(out)


def _int_ref(expr, d):
    """Exact integral over the unit triangle / tetrahedron by iterated
    antiderivatives (sympy polynomials), innermost variable xi first."""
    def integ(e, var, upper):
        F = sp.Poly(e, var).integrate()
        return sp.expand(F.as_expr().subs(var, upper) - F.as_expr().subs(var, 0))
    if d == 2:
        return integ(integ(expr, xi, 1 - eta), eta, 1)
    return integ(integ(integ(expr, xi, 1 - eta - zeta), eta, 1 - zeta), zeta, 1)


def test_basis_size_matches_paper_dof_counts():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "dof_counts.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for r in rows:
        d, M, ncells, dof = map(int, r[:4])
        assert ncells * B.n_basis(M, d) == dof


def test_basis_size_small_cases():
    assert [B.n_basis(M, 2) for M in range(5)] == [1, 3, 6, 10, 15]
    assert [B.n_basis(M, 3) for M in range(5)] == [1, 4, 10, 20, 35]


def test_linear_functions_closed_form():
    # P_1^(0,0)(a) (1-b)/2 = 2 xi + eta - 1 and P_1^(1,0)(b) = 3 eta - 1 (hand derivation)
    P2 = B.dubiner_unnormalised(1, 2)
    assert _to_sympy(P2[0], 2) == 1
    assert _to_sympy(P2[1], 2) == sp.expand(2 * xi + eta - 1)
    assert _to_sympy(P2[2], 2) == sp.expand(3 * eta - 1)
    P3 = B.dubiner_unnormalised(1, 3)
    assert _to_sympy(P3[1], 3) == sp.expand(2 * xi + eta + zeta - 1)
    assert _to_sympy(P3[2], 3) == sp.expand(3 * eta + zeta - 1)
    assert _to_sympy(P3[3], 3) == sp.expand(4 * zeta - 1)
    # normalisation factors sqrt(6), sqrt(2) (2-D) and sqrt(10), sqrt(10/3), sqrt(5/3) (3-D)
    assert B.norm_scale_sq(1, 2) == (1, 6, 2)
    assert B.norm_scale_sq(1, 3) == (1, 10, Fraction(10, 3), Fraction(5, 3))


@pytest.mark.parametrize("d,M", [(2, 4), (3, 3)])
def test_orthogonality_by_symbolic_integration(d, M):
    P = [_to_sympy(p, d) for p in B.dubiner_unnormalised(M, d)]
    s2 = B.norm_scale_sq(M, d)
    vol = sp.Rational(1, math.factorial(d))
    n = len(P)
    rng = np.random.default_rng(1)
    pairs = [(l, l) for l in range(n)] + [tuple(sorted(rng.choice(n, 2, replace=False))) for _ in range(12)]
    for l, m in pairs:
        g = _int_ref(P[l] * P[m], d)
        if l == m:
            assert sp.Rational(s2[l].numerator, s2[l].denominator) * g == vol
        else:
            assert g == 0


def test_gram_diagonals_known_values():
    # int_{T_E} psi^2 of the unnormalised functions, derived by hand / sympy
    g2 = [Fraction(1, k) for k in (2, 12, 4, 30, 18, 6, 56, 40, 24, 8)]
    g3 = [Fraction(1, k) for k in (6, 60, 20, 10, 210, 126, 84, 42, 28, 14)]
    G2 = B.gram_unnormalised(3, 2)
    G3 = B.gram_unnormalised(2, 3)
    assert [G2[l][l] for l in range(10)] == g2
    assert [G3[l][l] for l in range(10)] == g3


@pytest.mark.parametrize("d,M", [(2, 4), (3, 4)])
def test_expansion_matches_collapsed_definition(d, M):
    """Monomial expansion == Jacobi products in collapsed coordinates (scipy)."""
    rng = np.random.default_rng(3)
    pts = rng.dirichlet(np.ones(d + 1), size=50)[:, 1:]
    vals = B.evaluate(M, d, pts)
    s = [math.sqrt(x) for x in B.norm_scale_sq(M, d)]
    for l, ind in enumerate(B.index_list(M, d)):
        if d == 2:
            p, q = ind
            X, Y = pts[:, 0], pts[:, 1]
            a = 2 * X / (1 - Y) - 1
            b = 2 * Y - 1
            ref = eval_jacobi(p, 0, 0, a) * ((1 - b) / 2) ** p * eval_jacobi(q, 2 * p + 1, 0, b)
        else:
            p, q, r = ind
            X, Y, Z = pts[:, 0], pts[:, 1], pts[:, 2]
            a = 2 * X / (1 - Y - Z) - 1
            b = 2 * Y / (1 - Z) - 1
            c = 2 * Z - 1
            ref = (eval_jacobi(p, 0, 0, a) * ((1 - b) / 2) ** p * eval_jacobi(q, 2 * p + 1, 0, b)
                   * ((1 - c) / 2) ** (p + q) * eval_jacobi(r, 2 * p + 2 * q + 2, 0, c))
        np.testing.assert_allclose(vals[:, l], s[l] * ref, rtol=1e-11, atol=1e-11)
    assert np.allclose(vals[:, 0], 1.0)


@pytest.mark.parametrize("d,M", [(2, 3), (3, 2)])
def test_sigma_quadratic_form_by_symbolic_derivatives(d, M):
    """c^T Sigma c == sum over distinct alpha, 1<=|alpha|<=M, of int (d^alpha P)^2."""
    syms = (xi, eta, zeta)[:d]
    P = [_to_sympy(p, d) for p in B.dubiner_unnormalised(M, d)]
    s = [sp.sqrt(sp.Rational(x.numerator, x.denominator)) for x in B.norm_scale_sq(M, d)]
    S = B.sigma_matrix(M, d)
    rng = np.random.default_rng(11)
    for _ in range(2):
        c = rng.integers(-3, 4, size=len(P))
        poly = sp.expand(sum(int(c[l]) * s[l] * P[l] for l in range(len(P))))
        tot = 0
        for n in range(1, M + 1):
            for alpha in itertools.product(range(n + 1), repeat=d):
                if sum(alpha) != n:
                    continue
                dp = poly
                for a in range(d):
                    dp = sp.diff(dp, syms[a], alpha[a])
                tot += _int_ref(sp.expand(dp * dp), d)
        assert abs(float(c @ S @ c) - float(tot)) <= 1e-12 * max(1.0, abs(float(tot)))


def test_sigma_linear_closed_form():
    """For a linear P with reference gradient g: sigma = |T_E| |g|^2."""
    rng = np.random.default_rng(5)
    for d in (2, 3):
        S = B.sigma_matrix(3, d)
        for _ in range(5):
            g = rng.normal(size=d)
            # coefficients of the linear function g . (xi - barycentre) in the orthonormal basis
            pts = rng.dirichlet(np.ones(d + 1), size=d + 3)[:, 1:]
            vals = B.evaluate(3, d, pts)[:, 1:d + 1]
            target = (pts - 1.0 / (d + 1)) @ g
            c, *_ = np.linalg.lstsq(vals, target, rcond=None)
            full = np.zeros(S.shape[0])
            full[1:d + 1] = c
            assert abs(full @ S @ full - g @ g / math.factorial(d)) < 1e-12 * (g @ g)
    assert np.all(B.sigma_matrix(2, 2)[0] == 0) and np.all(B.sigma_matrix(2, 3)[:, 0] == 0)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("deg", [1, 2, 3, 4, 5])
def test_collapsed_quadrature_exact(d, deg):
    pts, w = collapsed_rule(d, deg)
    assert abs(w.sum() - 1.0 / math.factorial(d)) < 1e-15
    for e in itertools.product(range(deg + 1), repeat=d):
        if sum(e) > deg:
            continue
        val = np.sum(w * np.prod(pts ** np.array(e), axis=1))
        exact = math.prod(math.factorial(k) for k in e) / math.factorial(sum(e) + d)
        assert abs(val - exact) < 1e-15
