"""Cell geometry in each cell's own reference frame -- oracle side.

Sec. 2 (eq. xietaTransf) maps cell T_i affinely onto the reference simplex
T_E with its first vertex at the origin: x = X_0 + J xi, J = [X_1 - X_0 | ...
| X_d - X_0].  Cell averages are defined by eq. cellaverage.

Periodic meshes (the paper's convergence tests use periodic boundaries; it
does not describe how stencil geometry crosses the wrap) are read with the
minimum-image convention, per periodic axis of length L:
    mi(delta) = delta - L * floor(delta / L + 0.5)
* a cell's vertices are unwrapped around its first vertex,
  X_k := X_0 + mi(X_k - X_0);
* its barycentre is (X_0 + ... + X_d) / (d + 1), summed left to right;
* a neighbour j is seen from cell i at offset mi(c_j - c_i) from c_i, i.e.
  all of j's unwrapped vertices are moved by mi(c_j - c_i) - (c_j - c_i).

Every floating-point formula that decides an integer table (barycentres,
offsets, squared distances, barycentric coordinates) is written out here
operation by operation on Python floats, so its rounding is fixed.
"""
from __future__ import annotations

import math

import numpy as np


def mi(delta: float, L: float) -> float:
    """Minimum-image offset along one axis (identity when L == 0)."""
    if L == 0.0:
        return delta
    return delta - L * math.floor(delta / L + 0.5)


class Geometry:
    """Per-cell unwrapped vertices and barycentres of a mesh (Python floats)."""

    def __init__(self, vertices: np.ndarray, cells: np.ndarray, box):
        self.d = int(vertices.shape[1])
        self.box = tuple(float(b) for b in box)
        self.V = vertices.astype(np.float64)
        self.C = cells.astype(np.int64)
        self._verts = {}
        self._cent = {}

    def cell_vertices(self, i: int):
        """Unwrapped vertex coordinates of cell i: list of d+1 tuples."""
        v = self._verts.get(i)
        if v is not None:
            return v
        d = self.d
        ids = self.C[i]
        X0 = [float(self.V[ids[0], a]) for a in range(d)]
        out = [tuple(X0)]
        for k in range(1, d + 1):
            Xk = [float(self.V[ids[k], a]) for a in range(d)]
            out.append(tuple(X0[a] + mi(Xk[a] - X0[a], self.box[a]) for a in range(d)))
        self._verts[i] = out
        return out

    def centroid(self, i: int):
        c = self._cent.get(i)
        if c is not None:
            return c
        X = self.cell_vertices(i)
        d = self.d
        out = []
        for a in range(d):
            s = X[0][a]
            for k in range(1, d + 1):
                s = s + X[k][a]
            out.append(s / (d + 1))
        c = tuple(out)
        self._cent[i] = c
        return c

    def offset(self, i: int, j: int):
        """mi(c_j - c_i) per axis."""
        ci = self.centroid(i)
        cj = self.centroid(j)
        return tuple(mi(cj[a] - ci[a], self.box[a]) for a in range(self.d))

    def dist2(self, i: int, j: int) -> float:
        o = self.offset(i, j)
        s = o[0] * o[0]
        for a in range(1, self.d):
            s = s + o[a] * o[a]
        return s

    def vertices_in_frame_of(self, i: int, j: int) -> np.ndarray:
        """Cell j's unwrapped vertices translated next to cell i [d+1, d]."""
        ci = self.centroid(i)
        cj = self.centroid(j)
        o = self.offset(i, j)
        shift = [o[a] - (cj[a] - ci[a]) for a in range(self.d)]
        X = np.array(self.cell_vertices(j), dtype=np.float64)
        return X + np.array(shift)[None, :]

    def jacobian(self, i: int) -> np.ndarray:
        X = np.array(self.cell_vertices(i), dtype=np.float64)
        return (X[1:] - X[0]).T            # columns X_k - X_0


def det_columns(W):
    """Determinant of [W_1 - W_0 | ... | W_d - W_0] by the explicit cofactor formula.

    2-D: u_x v_y - v_x u_y.
    3-D: u_x (v_y w_z - v_z w_y) - u_y (v_x w_z - v_z w_x) + u_z (v_x w_y - v_y w_x).
    """
    d = len(W) - 1
    if d == 2:
        ux = W[1][0] - W[0][0]
        uy = W[1][1] - W[0][1]
        vx = W[2][0] - W[0][0]
        vy = W[2][1] - W[0][1]
        return ux * vy - vx * uy
    ux = W[1][0] - W[0][0]
    uy = W[1][1] - W[0][1]
    uz = W[1][2] - W[0][2]
    vx = W[2][0] - W[0][0]
    vy = W[2][1] - W[0][1]
    vz = W[2][2] - W[0][2]
    wx = W[3][0] - W[0][0]
    wy = W[3][1] - W[0][1]
    wz = W[3][2] - W[0][2]
    return ux * (vy * wz - vz * wy) - uy * (vx * wz - vz * wx) + uz * (vx * wy - vy * wx)


def barycentric(X, p):
    """Barycentric coordinates of point p w.r.t. the simplex X (list of d+1 points).

    b_m = det(X with vertex m replaced by p) / det(X).
    """
    D = det_columns(X)
    out = []
    for m in range(len(X)):
        W = list(X)
        W[m] = p
        out.append(det_columns(W) / D)
    return out
