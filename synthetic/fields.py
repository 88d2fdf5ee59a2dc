"""Seeded analytic fields and their cell averages (the reconstruction's input).

A cell average is the integral of a field over the cell divided by its volume
(Sec. 2, eq. cellaverage).  Here it is evaluated with quadrature rules that
belong to this generator only:

* triangles: the 7-point degree-5 Radon rule (centroid plus two orbits of
  three points with coordinates (6 -+ sqrt 15)/21);
* tetrahedra (and triangles when more than degree 5 is asked for): a conical
  product of Gauss-Jacobi rules (Stroud), exact to degree 2m-1 with m points
  per collapsed direction.

A field is a callable ``f(x) -> array [n_vars, n_points]`` of physical
coordinates ``x`` with shape [dim, n_points].  On a periodic mesh the points
are wrapped into the box before the call, so fields with jumps are defined on
[0,1)^d.  Polynomial fields are meant for non-periodic meshes.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import roots_jacobi

from .meshes import SimplexMesh

GAMMA = 1.4


# ----------------------------------------------------------------- quadrature
def _radon7():
    s = math.sqrt(15.0)
    a1 = (6.0 - s) / 21.0
    a2 = (6.0 + s) / 21.0
    w1 = (155.0 - s) / 1200.0
    w2 = (155.0 + s) / 1200.0
    bary = [(1 / 3, 1 / 3, 1 / 3)]
    wts = [9.0 / 40.0]
    for a, w in ((a1, w1), (a2, w2)):
        b = 1.0 - 2.0 * a
        bary += [(b, a, a), (a, b, a), (a, a, b)]
        wts += [w, w, w]
    return np.array(bary), np.array(wts)


def _gj01(m, alpha):
    """Gauss-Jacobi nodes/weights on [0,1] for the weight (1-t)^alpha."""
    x, w = roots_jacobi(m, alpha, 0.0)
    return (x + 1.0) / 2.0, w / 2.0 ** (alpha + 1.0)


def _conical(dim, m):
    """Barycentric points and weights (sum 1) of a Stroud conical product rule."""
    if dim == 2:
        a, wa = _gj01(m, 0.0)
        b, wb = _gj01(m, 1.0)
        A, B = np.meshgrid(a, b, indexing="ij")
        W = np.outer(wa, wb)
        eta = B
        xi = A * (1.0 - B)
        lam = np.stack([1.0 - xi - eta, xi, eta], axis=-1).reshape(-1, 3)
        w = W.ravel() * 2.0            # divide by |T_E| = 1/2
        return lam, w
    a, wa = _gj01(m, 0.0)
    b, wb = _gj01(m, 1.0)
    c, wc = _gj01(m, 2.0)
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    W = wa[:, None, None] * wb[None, :, None] * wc[None, None, :]
    zeta = C
    eta = B * (1.0 - C)
    xi = A * (1.0 - B) * (1.0 - C)
    lam = np.stack([1.0 - xi - eta - zeta, xi, eta, zeta], axis=-1).reshape(-1, 4)
    w = W.ravel() * 6.0                # divide by |T_E| = 1/6
    return lam, w


def averaging_rule(dim: int, degree: int = 5):
    """(barycentric points [q, dim+1], weights [q] summing to 1), exact to ``degree``."""
    if dim == 2 and degree <= 5:
        return _radon7()
    m = max(1, (degree + 2) // 2)
    return _conical(dim, m)


def cell_averages(mesh: SimplexMesh, fn, degree: int = 5, chunk: int = 1 << 16) -> np.ndarray:
    """Cell averages [n_vars, n_cells] of the field ``fn`` over every cell."""
    lam, w = averaging_rule(mesh.dim, degree)
    out = None
    for s in range(0, mesh.n_cells, chunk):
        X = _unwrapped_cell_vertices_slice(mesh, s, min(mesh.n_cells, s + chunk))
        pts = np.einsum("qv,cvd->dcq", lam, X)           # [dim, cells, q]
        for a, L in enumerate(mesh.box):
            if L:
                pts[a] = pts[a] - L * np.floor(pts[a] / L)
        vals = fn(pts.reshape(mesh.dim, -1))            # [nv, cells*q]
        vals = np.asarray(vals, dtype=np.float64).reshape(vals.shape[0], X.shape[0], -1)
        avg = vals @ w
        if out is None:
            out = np.empty((vals.shape[0], mesh.n_cells), dtype=np.float64)
        out[:, s:s + X.shape[0]] = avg
    return out


def _unwrapped_cell_vertices_slice(mesh, s, e):
    X = mesh.vertices[mesh.cells[s:e].astype(np.int64)]
    for a, L in enumerate(mesh.box):
        if L:
            dx = X[:, 1:, a] - X[:, :1, a]
            X[:, 1:, a] = X[:, :1, a] + dx - L * np.round(dx / L)
    return X


# ----------------------------------------------------------------- fields
def euler2d_sod_circle(x):
    """Four Euler conserved variables (rho, rho u, rho v, E), gamma = 1.4.

    Sod states (rho, p) = (1, 1) inside the circle of radius 0.3 about
    (0.5, 0.5) and (0.125, 0.1) outside, times a smooth sine perturbation of
    the density; small sine velocities.
    """
    X, Y = x[0], x[1]
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    inside = r2 < 0.09
    s = 1.0 + 0.05 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    rho = np.where(inside, 1.0, 0.125) * s
    p = np.where(inside, 1.0, 0.1)
    u = 0.05 * np.sin(2 * np.pi * Y)
    v = 0.05 * np.sin(2 * np.pi * X)
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack([rho, rho * u, rho * v, E])


class smooth_fourier_field:
    """Seeded smooth periodic scalar fields: sums of ``modes`` plane waves.

    Each of the ``n`` fields is sum_m a_m sin(2 pi k_m . x + phi_m) with
    integer wavevectors |k_m|_inf <= kmax, sum |a_m| = 1, so |f| <= 1.
    """

    def __init__(self, dim, n, seed, modes=8, kmax=4):
        rng = np.random.default_rng(seed)
        self.k = rng.integers(-kmax, kmax + 1, size=(n, modes, dim))
        zero = np.all(self.k == 0, axis=-1)
        self.k[zero, 0] = 1
        a = rng.uniform(0.2, 1.0, size=(n, modes))
        self.a = a / a.sum(axis=1, keepdims=True)
        self.phi = rng.uniform(0, 2 * np.pi, size=(n, modes))

    def __call__(self, x):
        ph = 2 * np.pi * np.einsum("nmd,dp->nmp", self.k.astype(np.float64), x)
        return np.einsum("nm,nmp->np", self.a, np.sin(ph + self.phi[:, :, None]))


def mhd2d_fourier_jump(seed):
    """Nine ideal-MHD-shaped conserved variables on [0,1)^2.

    (rho, rho u, rho v, rho w, E, Bx, By, Bz, psi) with smooth seeded
    8-mode Fourier perturbations of every primitive variable and a planar
    jump at x = 0.5 with density ratio 10 (the periodic wrap makes x = 0 a
    second jump).  rho and p stay positive.
    """
    F = smooth_fourier_field(2, 9, seed, modes=8, kmax=4)

    def fn(x):
        f = F(x)
        left = x[0] < 0.5
        rho = np.where(left, 10.0, 1.0) * (1.0 + 0.2 * f[0])
        p = np.where(left, 10.0, 1.0) * (1.0 + 0.2 * f[4])
        u, v, w = 0.1 * f[1], 0.1 * f[2], 0.1 * f[3]
        bx, by, bz = 0.75 + 0.1 * f[5], 0.5 + 0.1 * f[6], 0.1 * f[7]
        psi = 0.01 * f[8]
        E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v + w * w) + 0.5 * (bx * bx + by * by + bz * bz)
        return np.stack([rho, rho * u, rho * v, rho * w, E, bx, by, bz, psi])
    return fn


def euler3d_blast(seed):
    """Five Euler conserved variables: spherical blast plus smooth perturbation.

    p = 1 for |x - c| < 0.25 and 0.1 outside (c = cube centre), rho = 1
    perturbed by 5 %, small smooth velocities.
    """
    F = smooth_fourier_field(3, 4, seed, modes=8, kmax=3)

    def fn(x):
        f = F(x)
        r2 = (x[0] - 0.5) ** 2 + (x[1] - 0.5) ** 2 + (x[2] - 0.5) ** 2
        p = np.where(r2 < 0.0625, 1.0, 0.1)
        rho = 1.0 + 0.05 * f[0]
        u, v, w = 0.05 * f[1], 0.05 * f[2], 0.05 * f[3]
        E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
        return np.stack([rho, rho * u, rho * v, rho * w, E])
    return fn


def smooth_plus_jump(dim, n_vars, seed):
    """Random smooth 8-mode fields plus one random planar or spherical jump."""
    rng = np.random.default_rng(seed)
    F = smooth_fourier_field(dim, n_vars, seed + 1, modes=8, kmax=3)
    planar = bool(rng.integers(0, 2))
    normal = rng.normal(size=dim)
    normal /= np.linalg.norm(normal)
    centre = rng.uniform(0.3, 0.7, size=dim)
    radius = rng.uniform(0.15, 0.3)
    base = rng.uniform(0.5, 2.0, size=n_vars)
    jump = rng.uniform(0.5, 4.0, size=n_vars)

    def fn(x):
        if planar:
            side = np.einsum("d,dp->p", normal, x - centre[:, None]) < 0.0
        else:
            side = np.sum((x - centre[:, None]) ** 2, axis=0) < radius * radius
        return base[:, None] * (1.0 + 0.1 * F(x)) + np.where(side, jump[:, None], 0.0)
    return fn


# ----------------------------------------------------------------- polynomials
def _exponents(dim, degree):
    out = []
    for n in range(degree + 1):
        if dim == 2:
            for a in range(n, -1, -1):
                out.append((a, n - a))
        else:
            for a in range(n, -1, -1):
                for b in range(n - a, -1, -1):
                    out.append((a, b, n - a - b))
    return out


def random_polynomial(dim, degree, n_vars, seed, centre=0.5):
    """Seeded random polynomials of total degree <= ``degree`` (one per variable).

    Returned as (exponents, coefficients [n_vars, n_terms], centre); the
    polynomial is sum_t c_t prod_a (x_a - centre)^e_ta.
    """
    rng = np.random.default_rng(seed)
    ex = _exponents(dim, degree)
    coef = rng.normal(size=(n_vars, len(ex)))
    return ex, coef, centre


def polynomial_field(poly):
    ex, coef, centre = poly

    def fn(x):
        y = x - centre
        terms = np.stack([np.prod([y[a] ** e[a] for a in range(len(e))], axis=0) for e in ex])
        return coef @ terms
    return fn


def workload_fields(mesh: SimplexMesh, kind: str, seed: int) -> np.ndarray:
    """Cell averages [n_vars, n_cells] for the named synthetic state."""
    if kind == "euler2d_sod":
        return cell_averages(mesh, euler2d_sod_circle, 5)
    if kind == "mhd2d":
        return cell_averages(mesh, mhd2d_fourier_jump(seed), 5)
    # tetrahedra: an 8-point degree-3 conical rule keeps million-cell inputs cheap
    deg = 5 if mesh.dim == 2 else 3
    if kind == "euler3d_blast":
        return cell_averages(mesh, euler3d_blast(seed), deg)
    if kind.startswith("smooth_jump"):
        nv = int(kind.split(":")[1]) if ":" in kind else mesh.dim + 2
        return cell_averages(mesh, smooth_plus_jump(mesh.dim, nv, seed), deg)
    raise ValueError(f"unknown field kind {kind!r}")
