"""Orthonormal Dubiner basis on the reference simplex and the universal
oscillation-indicator matrix -- oracle side (test infrastructure only).

Sec. 2.1 (eq. recpolydef) expands every reconstruction polynomial in an
orthogonal Dubiner-type basis psi_l(xi) on the reference element T_E (unit
triangle / unit tetrahedron, Fig. refSystem).  The paper names the family but
prints no formula, normalisation or order; the reading used here is:

* collapsed-coordinate Dubiner/Koornwinder functions
    2-D: psi_pq = P_p^(0,0)(a) ((1-b)/2)^p P_q^(2p+1,0)(b),
         a = 2 xi/(1-eta) - 1, b = 2 eta - 1;
    3-D: psi_pqr = P_p^(0,0)(a) ((1-b)/2)^p P_q^(2p+1,0)(b) ((1-c)/2)^(p+q)
                   P_r^(2p+2q+2,0)(c),
         a = 2 xi/(1-eta-zeta) - 1, b = 2 eta/(1-zeta) - 1, c = 2 zeta - 1;
* normalised so that (1/|T_E|) int_{T_E} psi_l psi_m = delta_lm (hence
  psi_1 = 1 and every other psi has zero mean on T_E);
* ordered by total degree, then p descending, then q descending.

Here every psi is expanded *exactly* into monomials xi^a eta^b (zeta^c) with
rational coefficients (``fractions.Fraction``): the collapsed factors combine
into the polynomials (2 xi + eta - 1), (1 - eta), ... so no singular division
is ever evaluated.  Integrals over T_E of monomials are the closed form
a! b! c! / (a+b+c+d)!.

The oscillation-indicator matrix of Sec. 2.1 (the sigma_s definition) is
    Sigma_lm = sum over distinct multi-indices alpha, 1 <= |alpha| <= M, of
               int_{T_E} d^alpha psi_l  d^alpha psi_m,
computed here exactly in rationals for the unnormalised functions and then
scaled by the normalisation factors.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr
from functools import lru_cache

import numpy as np


def n_basis(M: int, d: int) -> int:
    """Number of basis functions, eq. cwenoM: (1/d!) prod_{l=1..d} (M + l)."""
    num = 1
    for l in range(1, d + 1):
        num *= (M + l)
    return num // math.factorial(d)


# ------------------------------------------------------------ polynomial algebra
# A polynomial in d variables is a dict {exponent tuple: Fraction}.
def _padd(a, b):
    out = dict(a)
    for k, v in b.items():
        out[k] = out.get(k, Fr(0)) + v
    return {k: v for k, v in out.items() if v != 0}


def _pmul(a, b):
    out = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, Fr(0)) + va * vb
    return {k: v for k, v in out.items() if v != 0}


def _pscale(a, c):
    return {k: v * c for k, v in a.items() if v * c != 0}


def _ppow(a, n, d):
    out = {(0,) * d: Fr(1)}
    for _ in range(n):
        out = _pmul(out, a)
    return out


def _lin(d, const, *coeffs):
    """const + sum_a coeffs[a] * x_a as a polynomial."""
    out = {}
    if const:
        out[(0,) * d] = Fr(const)
    for a, c in enumerate(coeffs):
        if c:
            e = [0] * d
            e[a] = 1
            out[tuple(e)] = Fr(c)
    return out


def _jacobi_coeffs(n: int, alpha: int):
    """Power-series coefficients (in x) of the Jacobi polynomial P_n^(alpha,0)(x).

    Uses the explicit sum P_n^(a,b)(x) = sum_s C(n+a, n-s) C(n+b, s)
    ((x-1)/2)^s ((x+1)/2)^(n-s) with b = 0.
    """
    xm = {(0,): Fr(-1, 2), (1,): Fr(1, 2)}    # (x-1)/2
    xp = {(0,): Fr(1, 2), (1,): Fr(1, 2)}     # (x+1)/2
    acc = {}
    for s in range(n + 1):
        c = Fr(math.comb(n + alpha, n - s) * math.comb(n, s))
        term = _pscale(_pmul(_ppow(xm, s, 1), _ppow(xp, n - s, 1)), c)
        acc = _padd(acc, term)
    out = [Fr(0)] * (n + 1)
    for (k,), v in acc.items():
        out[k] = v
    return out


def _compose_collapsed(coeffs, top, bottom, deg, d):
    """sum_k coeffs[k] * top^k * bottom^(deg-k): P(a) * bottom^deg with a*bottom = top."""
    out = {}
    for k, c in enumerate(coeffs):
        if c == 0:
            continue
        term = _pmul(_ppow(top, k, d), _ppow(bottom, deg - k, d))
        out = _padd(out, _pscale(term, c))
    return out


def _compose(coeffs, lin, d):
    """P(lin) for a univariate coefficient list and a polynomial argument."""
    out = {}
    for k, c in enumerate(coeffs):
        if c == 0:
            continue
        out = _padd(out, _pscale(_ppow(lin, k, d), c))
    return out


def index_list(M: int, d: int):
    """The (p, q[, r]) indices of the basis in order (degree, p desc, q desc)."""
    idx = []
    for n in range(M + 1):
        for p in range(n, -1, -1):
            if d == 2:
                idx.append((p, n - p))
            else:
                for q in range(n - p, -1, -1):
                    idx.append((p, q, n - p - q))
    return idx


@lru_cache(maxsize=None)
def dubiner_unnormalised(M: int, d: int):
    """Exact monomial expansions of the unnormalised Dubiner functions."""
    polys = []
    for ind in index_list(M, d):
        if d == 2:
            p, q = ind
            t1 = _compose_collapsed(_jacobi_coeffs(p, 0), _lin(2, -1, 2, 1), _lin(2, 1, 0, -1), p, 2)
            t2 = _compose(_jacobi_coeffs(q, 2 * p + 1), _lin(2, -1, 0, 2), 2)
            polys.append(_pmul(t1, t2))
        else:
            p, q, r = ind
            t1 = _compose_collapsed(_jacobi_coeffs(p, 0), _lin(3, -1, 2, 1, 1), _lin(3, 1, 0, -1, -1), p, 3)
            t2 = _compose_collapsed(_jacobi_coeffs(q, 2 * p + 1), _lin(3, -1, 0, 2, 1), _lin(3, 1, 0, 0, -1), q, 3)
            t3 = _compose(_jacobi_coeffs(r, 2 * p + 2 * q + 2), _lin(3, -1, 0, 0, 2), 3)
            polys.append(_pmul(_pmul(t1, t2), t3))
    return tuple(polys)


def monomial_integral(e) -> Fr:
    """int over T_E of prod x_a^e_a  =  prod(e_a!) / (sum e + d)!."""
    num = 1
    for k in e:
        num *= math.factorial(k)
    return Fr(num, math.factorial(sum(e) + len(e)))


def integrate(poly) -> Fr:
    return sum((c * monomial_integral(e) for e, c in poly.items()), Fr(0))


def ref_volume(d: int) -> Fr:
    return Fr(1, math.factorial(d))


@lru_cache(maxsize=None)
def gram_unnormalised(M: int, d: int):
    """Exact Gram matrix int_{T_E} psi_l psi_m of the unnormalised functions."""
    P = dubiner_unnormalised(M, d)
    n = len(P)
    G = [[Fr(0)] * n for _ in range(n)]
    for l in range(n):
        for m in range(l, n):
            G[l][m] = G[m][l] = integrate(_pmul(P[l], P[m]))
    return G


@lru_cache(maxsize=None)
def norm_scale_sq(M: int, d: int):
    """Exact s_l^2 = |T_E| / int psi_l^2, so that s_l psi_l is orthonormal."""
    G = gram_unnormalised(M, d)
    return tuple(ref_volume(d) / G[l][l] for l in range(len(G)))


def _sqrt_frac(f: Fr) -> np.longdouble:
    return np.sqrt(np.longdouble(f.numerator) / np.longdouble(f.denominator))


@lru_cache(maxsize=None)
def _eval_tables(M: int, d: int):
    P = dubiner_unnormalised(M, d)
    s = [_sqrt_frac(x) for x in norm_scale_sq(M, d)]
    exps = sorted({e for p in P for e in p})
    C = np.zeros((len(P), len(exps)), dtype=np.longdouble)
    col = {e: k for k, e in enumerate(exps)}
    for l, p in enumerate(P):
        for e, c in p.items():
            C[l, col[e]] = (np.longdouble(c.numerator) / np.longdouble(c.denominator)) * s[l]
    return np.array(exps, dtype=np.int64), C


def evaluate(M: int, d: int, pts: np.ndarray) -> np.ndarray:
    """psi_l at reference points: pts [n, d] -> values [n, n_basis] (float64).

    Evaluated from the exact monomial expansion in extended precision.
    """
    exps, C = _eval_tables(M, d)
    X = np.asarray(pts, dtype=np.longdouble)
    mon = np.ones((X.shape[0], exps.shape[0]), dtype=np.longdouble)
    for a in range(d):
        mon *= X[:, a:a + 1] ** exps[None, :, a]
    return (mon @ C.T).astype(np.float64)


def _derivative(poly, alpha):
    out = {}
    for e, c in poly.items():
        coef = c
        ne = list(e)
        ok = True
        for a, k in enumerate(alpha):
            if e[a] < k:
                ok = False
                break
            for t in range(k):
                coef *= (e[a] - t)
            ne[a] = e[a] - k
        if ok and coef != 0:
            out[tuple(ne)] = out.get(tuple(ne), Fr(0)) + coef
    return out


def _multi_indices(d, lo, hi):
    out = []
    for n in range(lo, hi + 1):
        if d == 2:
            for a in range(n, -1, -1):
                out.append((a, n - a))
        else:
            for a in range(n, -1, -1):
                for b in range(n - a, -1, -1):
                    out.append((a, b, n - a - b))
    return out


@lru_cache(maxsize=None)
def sigma_unnormalised(M: int, d: int):
    """Exact Sigma_lm for the unnormalised functions (rationals)."""
    P = dubiner_unnormalised(M, d)
    n = len(P)
    S = [[Fr(0)] * n for _ in range(n)]
    for alpha in _multi_indices(d, 1, M):
        D = [_derivative(p, alpha) for p in P]
        for l in range(n):
            if not D[l]:
                continue
            for m in range(l, n):
                if not D[m]:
                    continue
                v = integrate(_pmul(D[l], D[m]))
                S[l][m] += v
                if m != l:
                    S[m][l] += v
    return S


@lru_cache(maxsize=None)
def sigma_matrix(M: int, d: int) -> np.ndarray:
    """Universal oscillation-indicator matrix of the orthonormal basis (float64)."""
    S = sigma_unnormalised(M, d)
    s = [_sqrt_frac(x) for x in norm_scale_sq(M, d)]
    n = len(S)
    out = np.zeros((n, n), dtype=np.float64)
    for l in range(n):
        for m in range(n):
            out[l, m] = float(np.longdouble(S[l][m].numerator) / np.longdouble(S[l][m].denominator) * s[l] * s[m])
    return out
