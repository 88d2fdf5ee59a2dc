"""Collapsed (Duffy) Gauss-Legendre rules on the reference simplex -- oracle side.

Sec. 2.1 evaluates the cell-average integrals of the least-squares problem
(eq. CWENO:Popt) in reference coordinates with Gaussian quadrature of suitable
order.  The oracle uses a tensor Gauss-Legendre rule on [0,1]^d mapped to T_E
by the collapsing map
    2-D: xi = u (1 - v),             eta = v,               |J| = (1 - v)
    3-D: xi = u (1 - v)(1 - w),      eta = v (1 - w),  zeta = w,
                                                            |J| = (1 - v)(1 - w)^2
with plain Legendre points (the Jacobian is carried in the weights), exact
for polynomials of total degree <= ``degree``.
"""
from __future__ import annotations

import numpy as np


def collapsed_rule(d: int, degree: int):
    """Points [q, d] in T_E and weights [q] summing to |T_E| = 1/d!."""
    n = max(1, (degree + d + 1) // 2)          # 2n-1 >= degree + (d-1)
    x, w = np.polynomial.legendre.leggauss(n)
    t = (x + 1.0) / 2.0
    wt = w / 2.0
    if d == 2:
        U, V = np.meshgrid(t, t, indexing="ij")
        W = np.outer(wt, wt) * (1.0 - V)
        pts = np.stack([U * (1.0 - V), V], axis=-1).reshape(-1, 2)
        return pts, W.ravel()
    U, V, Wc = np.meshgrid(t, t, t, indexing="ij")
    W = wt[:, None, None] * wt[None, :, None] * wt[None, None, :] * (1.0 - V) * (1.0 - Wc) ** 2
    pts = np.stack([U * (1.0 - V) * (1.0 - Wc), V * (1.0 - Wc), Wc], axis=-1).reshape(-1, 3)
    return pts, W.ravel()
