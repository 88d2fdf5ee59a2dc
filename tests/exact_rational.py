"""Exact-rational brute force of the CWENO and classical WENO pipelines on
tiny meshes (shared by the oracle's brute-force pins; not collected).

Independent of the oracle's arithmetic: polynomials are kept in the monomial
basis of cell i's reference coordinates, stencil averages are integrated
exactly over each (dyadic-rational) simplex through barycentric monomial
integrals, every constrained least-squares polynomial (Sec. 2.1, eq.
CWENO:Popt) comes from the KKT system of the equality-constrained problem
solved by exact Gauss-Jordan elimination, the sectorial P1 systems (eq.
CWENO:Ps) likewise, and the indicators sum_alpha int (d^alpha P)^2, the
weights (eps = 1e-14 as an exact rational) and the blend are all exact.

Sector decisions are taken here too, from their definitions: a sector with
no cells is dropped, and so is one whose d x d system in the orthonormal
linear basis has 2-norm condition number above 1e10 (decided exactly from
the characteristic polynomial of B^T B); the linear weights of the kept
polynomials are then renormalised in rationals.
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import sympy

EPS = Fr(1, 10 ** 14)
COND_MAX = 10 ** 10

# squared normalisations of the orthonormal linear Dubiner functions, in the
# order of the unnormalised forms below (derived by exact integration over
# the reference simplex; pinned in the basis tests)
LIN_SCALE2 = {2: (Fr(6), Fr(2)), 3: (Fr(10), Fr(10, 3), Fr(5, 3))}


def lin_unnormalised(d, xi):
    """2-D: 2x+y-1, 3y-1; 3-D: 2x+y+z-1, 3y+z-1, 4z-1."""
    if d == 2:
        x, y = xi
        return [2 * x + y - 1, 3 * y - 1]
    x, y, z = xi
    return [2 * x + y + z - 1, 3 * y + z - 1, 4 * z - 1]


def exps_of(d, M):
    out = []
    for n in range(M + 1):
        for e in itertools.product(range(n + 1), repeat=d):
            if sum(e) == n:
                out.append(e)
    return out


def poly_mul(a, b):
    out = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, Fr(0)) + va * vb
    return out


def simplex_avg_monomial(Y, e):
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
            poly = poly_mul(poly, lin)
    tot = Fr(0)
    for K, c in poly.items():
        tot += c * Fr(math.factorial(d) * math.prod(math.factorial(k) for k in K), math.factorial(sum(K) + d))
    return tot


def solve(A, b):
    """Exact Gauss-Jordan with pivot search; A square list of lists.  None if singular."""
    n = len(A)
    M = [list(A[r]) + [b[r]] for r in range(n)]
    for c in range(n):
        p = next((r for r in range(c, n) if M[r][c] != 0), None)
        if p is None:
            return None
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[r][n] for r in range(n)]


def ref_integral(e):
    return Fr(math.prod(math.factorial(k) for k in e), math.factorial(sum(e) + len(e)))


def sigma_exact(coef, exps, d, M):
    """sum over distinct alpha, 1 <= |alpha| <= M, of int_{T_E} (d^alpha P)^2."""
    tot = Fr(0)
    for alpha in exps_of(d, M)[1:]:
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
        sq = poly_mul(der, der)
        tot += sum((c * ref_integral(k) for k, c in sq.items()), Fr(0))
    return tot


def cond_exceeds(L, d, cmax=COND_MAX):
    """True when B = L diag(c) (c_l^2 = LIN_SCALE2) is singular or has 2-norm
    condition number above ``cmax``.  The eigenvalues of B^T B are those of
    L^T L diag(c^2), a rational matrix: its characteristic polynomial is
    exact and its roots are isolated to 60 digits."""
    c2 = LIN_SCALE2[d]
    K = [[sum((L[k][a] * L[k][b] for k in range(d)), Fr(0)) * c2[b] for b in range(d)] for a in range(d)]
    Ms = sympy.Matrix(d, d, lambda a, b: sympy.Rational(K[a][b].numerator, K[a][b].denominator))
    if Ms.det() == 0:
        return True
    lam = sympy.symbols("lam")
    roots = sympy.Poly(Ms.charpoly(lam).as_expr(), lam).nroots(n=60)
    roots = sorted(sympy.re(r) for r in roots)
    return roots[-1] > cmax * cmax * roots[0]


def frac_vertices(o, i, j):
    return [[Fr(float(x)) for x in row] for row in o.geo.vertices_in_frame_of(i, j)]


class ExactCell:
    """Exact quantities of cell i of an oracle mesh ``o`` (a CwenoOracle)."""

    def __init__(self, o, i):
        self.o, self.i, self.d, self.M = o, i, o.d, o.M
        d = self.d
        self.exps = exps_of(d, self.M)
        self.Xi = [[Fr(float(x)) for x in row] for row in o.geo.cell_vertices(i)]
        J = [[self.Xi[k + 1][a] - self.Xi[0][a] for k in range(d)] for a in range(d)]
        cols = [solve(J, [Fr(int(r == c)) for r in range(d)]) for c in range(d)]
        self.Jinv = [[cols[c][r] for c in range(d)] for r in range(d)]
        self._rows = {}

    def to_ref(self, x):
        d = self.d
        y = [x[a] - self.Xi[0][a] for a in range(d)]
        return [sum((self.Jinv[r][a] * y[a] for a in range(d)), Fr(0)) for r in range(d)]

    def row(self, j):
        """Exact averages over cell j of every monomial of degree <= M in xi_i."""
        r = self._rows.get(j)
        if r is None:
            Y = [self.to_ref(v) for v in frac_vertices(self.o, self.i, j)]
            r = [simplex_avg_monomial(Y, e) for e in self.exps]
            self._rows[j] = r
        return r

    def barycentre_ref(self, j):
        Y = [self.to_ref(v) for v in frac_vertices(self.o, self.i, j)]
        return [sum((y[a] for y in Y), Fr(0)) / (self.d + 1) for a in range(self.d)]

    def constrained_lsq(self, S, q):
        """argmin ||A p - q||^2 s.t. (A p)_0 = q_0 over stencil S (S[0] = i), by KKT."""
        A = [self.row(j) for j in S]
        nm = len(self.exps)
        K = [[2 * sum((A[k][r] * A[k][c] for k in range(len(A))), Fr(0)) for c in range(nm)] + [A[0][r]]
             for r in range(nm)]
        K.append(A[0] + [Fr(0)])
        rhs = [2 * sum((A[k][r] * q[k] for k in range(len(A))), Fr(0)) for r in range(nm)] + [q[0]]
        return solve(K, rhs)[:nm]

    def sector_poly(self, sec, Qcol, cmax=COND_MAX):
        """Degree-1 polynomial matching the averages on the d+1 sector cells,
        or None when the sector is empty, singular or worse conditioned than
        ``cmax`` in the orthonormal linear basis."""
        if sec is None:
            return None
        L = [lin_unnormalised(self.d, self.barycentre_ref(j)) for j in sec[1:]]
        if cond_exceeds(L, self.d, cmax):
            return None
        lin = [t for t, e in enumerate(self.exps) if sum(e) <= 1]
        As = [[self.row(j)[t] for t in lin] for j in sec]
        ps = solve(As, [Fr(Qcol[j]) for j in sec])
        full = [Fr(0)] * len(self.exps)
        for t, v in zip(lin, ps):
            full[t] = v
        return full

    def value(self, coef, pt):
        return sum((coef[t] * math.prod(Fr(pt[a]) ** self.exps[t][a] for a in range(self.d))
                    for t in range(len(self.exps))), Fr(0))


def exact_cweno(o, i, Qcol, lam, sectors=None, sigma0_popt=False, r=4):
    """Exact CWENO of one variable at cell i.

    ``lam``: linear weights lambda_0..lambda_{d+1} (rationals, summing to 1);
    ``sectors``: sector lists (None = empty) -- default the oracle's tables.
    Returns dict(w, sigma, omega, alive, exps, cell)."""
    ec = ExactCell(o, i)
    d = ec.d
    S0, sec_o = o.stencils(i)
    secs = sec_o if sectors is None else sectors
    popt = ec.constrained_lsq(S0, [Fr(Qcol[j]) for j in S0])
    nm = len(ec.exps)
    polys, alive = [], []
    for sec in secs:
        p = ec.sector_poly(sec, Qcol)
        alive.append(p is not None)
        polys.append(p if p is not None else [Fr(0)] * nm)
    lam = [lam[0]] + [lam[s + 1] if alive[s] else Fr(0) for s in range(d + 1)]
    tot = sum(lam, Fr(0))
    lam = [x / tot for x in lam]
    p0 = [(popt[t] - sum((lam[s + 1] * polys[s][t] for s in range(d + 1)), Fr(0))) / lam[0] for t in range(nm)]
    allp = [p0] + polys
    sig = [sigma_exact(p, ec.exps, d, ec.M) for p in allp]
    if sigma0_popt:
        sig[0] = sigma_exact(popt, ec.exps, d, ec.M)
    wt = [lam[s] / (sig[s] + EPS) ** r for s in range(d + 2)]
    tot = sum(wt, Fr(0))
    om = [x / tot for x in wt]
    w = [sum((om[s] * allp[s][t] for s in range(d + 2)), Fr(0)) for t in range(nm)]
    return dict(w=w, sigma=sig, omega=om, alive=alive, exps=ec.exps, cell=ec, lam=lam)


def exact_weno(o, i, Qcol, lam_raw, r=4):
    """Exact classical WENO of one variable at cell i of a WenoOracle ``o``:
    every stencil's constrained least-squares polynomial of degree M, the
    raw linear weights ``lam_raw`` (one per stencil) restricted to the
    stencils that exist and renormalised, omega~ = lambda / (sigma+eps)^r."""
    ec = ExactCell(o.cw, i)
    st = o.stencils(i)
    polys, lam = [], []
    for S, l in zip(st, lam_raw):
        if S is None:
            polys.append(None)
            lam.append(Fr(0))
            continue
        polys.append(ec.constrained_lsq(S, [Fr(Qcol[j]) for j in S]))
        lam.append(l)
    tot = sum(lam, Fr(0))
    lam = [x / tot for x in lam]
    nm = len(ec.exps)
    polys = [p if p is not None else [Fr(0)] * nm for p in polys]
    sig = [sigma_exact(p, ec.exps, ec.d, ec.M) for p in polys]
    wt = [lam[s] / (sig[s] + EPS) ** r for s in range(len(polys))]
    tot = sum(wt, Fr(0))
    om = [x / tot for x in wt]
    w = [sum((om[s] * polys[s][t] for s in range(len(polys))), Fr(0)) for t in range(nm)]
    return dict(w=w, sigma=sig, omega=om, lam=lam, exps=ec.exps, cell=ec)


def point_values(ec, coef, pts):
    return [float(ec.value(coef, p)) for p in pts]
