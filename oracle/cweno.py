"""CWENO reconstruction on simplex meshes, written plainly in FP64 -- oracle side.

Follows Sec. 2.1 step by step, per cell i and for all variables at once:

1. Central stencil S_i^0 (eq. stencil) and the d+1 sectorial stencils.
2. Stencil averages A[k, l] = average over T_j(k) of psi_l(xi_i(x)), every
   integral in cell i's reference coordinates (eq. xietaTransf; Gaussian
   quadrature, here a collapsed Gauss-Legendre rule exact for degree M).
3. P_opt (eq. CWENO:Popt): least squares over the stencil averages subject to
   the own-cell average being matched exactly.  Solved generically by the
   null-space method: a Householder QR of the constraint row gives a basis
   of its null space, the remaining unconstrained problem goes to
   ``numpy.linalg.lstsq`` (SVD).  No use is made of the basis having zero
   mean.
4. Sectorial P1 polynomials (eq. CWENO:Ps): the square (d+1)x(d+1) average-
   matching system on each sector, ``numpy.linalg.solve``.
5. P0 = (P_opt - sum_s lambda_s P_s) / lambda_0 (eq. CWENO:P0).
6. sigma_s = p_s^T Sigma p_s with the universal matrix Sigma (Sec. 2.1).
7. omega~_s = lambda_s / (sigma_s + eps)^r, omega = omega~ / sum omega~
   (eqs. weights, weights2), w = sum_s omega_s P_s (eq. CWENO:Prec).

Readings where the paper is silent or inconsistent (all shared with the
library, stated once more in the project documentation):

* Linear weights must sum to one (Sec. 2.1 requires it for the linear
  combination to equal P_opt).  Default lambda_0 = 0.95 and (1-lambda_0)/(d+1)
  per sector; ``lambda0='paper'`` normalises the paper's pair (1e5 for the
  central stencil, 1 per sector) to lambda_0 = 1e5/(1e5+d+1).
* N_p = d+1 sectors, so d+2 polynomials enter the blend (the blend's
  summation index s runs over P_0 .. P_{d+1}).
* sigma_0 is the indicator of P_0 (the polynomial that carries omega_0);
  ``sigma0_from='popt'`` uses P_opt instead.
* Stencil size n_e = ceil(f * M_basis), f = d by default (Sec. 2.1).
* A sector that cannot be filled, or whose reduced d x d system has 2-norm
  condition number above 1e10, is dropped: its lambda is set to zero and the
  remaining linear weights are renormalised.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import basis as B
from .geometry import Geometry
from .quadrature import collapsed_rule
from .stencils import StencilError, central_stencil, face_neighbours, sector_stencils

SECTOR_COND_MAX = 1e10


@dataclass
class Options:
    degree: int = 2
    stencil_factor: float = 0.0       # 0 -> d (the paper's n_e = d * M_basis)
    lambda0: object = 0.95            # float, or 'paper'
    eps: float = 1e-14
    r: int = 4
    sector_rule: str = "cone"         # 'cone' (Sec. 2.1) or 'face'
    sigma0_from: str = "p0"           # 'p0' or 'popt'
    linear_weights: bool = False      # diagnostic: omega := lambda


def stencil_size(M: int, d: int, factor: float) -> int:
    f = float(d) if factor == 0.0 else float(factor)
    return int(math.ceil(f * B.n_basis(M, d)))


def linear_weights(d: int, lambda0) -> np.ndarray:
    """lambda_0 .. lambda_{d+1}, positive and summing to one."""
    if lambda0 == "paper":
        tot = 1e5 + (d + 1)
        return np.array([1e5 / tot] + [1.0 / tot] * (d + 1))
    l0 = float(lambda0)
    if not (0.0 < l0 < 1.0):
        raise ValueError("lambda0 must lie in (0, 1)")
    return np.array([l0] + [(1.0 - l0) / (d + 1)] * (d + 1))


class CwenoOracle:
    """Plain FP64 CWENO reconstruction of one mesh."""

    def __init__(self, vertices, cells, box, opts: Options, nbr=None, stencils=None):
        """``stencils``: optional fixed tables (central [n, n_e], sectors
        [n, d+1, d+1] with rows of -1 for unfilled sectors) used instead of
        selecting stencils on this geometry -- a moving mesh keeps the
        stencils of its connectivity while its vertices move, and only the
        reconstruction matrices change (Sec. 2.1 on ALE meshes)."""
        self.V = np.asarray(vertices, dtype=np.float64)
        self.Cells = np.asarray(cells, dtype=np.int64)
        self.d = int(self.V.shape[1])
        self.opts = opts
        self.M = int(opts.degree)
        self.nb = B.n_basis(self.M, self.d)
        self.n_e = stencil_size(self.M, self.d, opts.stencil_factor)
        self.geo = Geometry(self.V, self.Cells, box)
        self.nbr = face_neighbours(self.Cells) if nbr is None else nbr
        self.Sigma = B.sigma_matrix(self.M, self.d)
        self.qpts, self.qw = collapsed_rule(self.d, self.M)
        self.qw_avg = self.qw / self.qw.sum()
        self.lam = linear_weights(self.d, opts.lambda0)
        self._stencil_cache = {}
        self._fixed = None
        if stencils is not None:
            central, sectors = stencils
            self._fixed = (np.asarray(central, dtype=np.int64), np.asarray(sectors, dtype=np.int64))
            if self._fixed[0].shape != (self.Cells.shape[0], self.n_e):
                raise ValueError("fixed central stencils must be [n_cells, n_e]")

    # ------------------------------------------------------------ tables
    def stencils(self, i: int):
        """(central stencil list, list of d+1 sector lists or None)."""
        c = self._stencil_cache.get(i)
        if c is None and self._fixed is not None:
            S0 = [int(j) for j in self._fixed[0][i]]
            Ss = [None if row[0] < 0 else [int(j) for j in row] for row in self._fixed[1][i]]
            c = (S0, Ss)
            self._stencil_cache[i] = c
        if c is None:
            S0 = central_stencil(self.geo, self.nbr, i, self.n_e)
            Ss = sector_stencils(self.geo, self.nbr, i, self.opts.sector_rule)
            c = (S0, Ss)
            self._stencil_cache[i] = c
        return c

    # ------------------------------------------------------------ averages
    def stencil_averages(self, i: int, cells) -> np.ndarray:
        """A[k, l] = (1/|T_j|) int_{T_j} psi_l(xi_i(x)) dx for j = cells[k]."""
        d = self.d
        X0 = np.array(self.geo.cell_vertices(i)[0])
        Jinv = np.linalg.inv(self.geo.jacobian(i))
        lamq = np.concatenate([1.0 - self.qpts.sum(axis=1, keepdims=True), self.qpts], axis=1)
        pts = []
        for j in cells:
            Xj = self.geo.vertices_in_frame_of(i, j)               # [d+1, d]
            Y = (Xj - X0[None, :]) @ Jinv.T                        # vertices in xi_i
            pts.append(lamq @ Y)                                   # [q, d]
        P = np.concatenate(pts, axis=0)
        vals = B.evaluate(self.M, d, P).reshape(len(cells), len(self.qw), self.nb)
        return np.einsum("q,kql->kl", self.qw_avg, vals)

    # ------------------------------------------------------------ steps
    @staticmethod
    def constrained_lsq(A: np.ndarray, QS: np.ndarray) -> np.ndarray:
        """argmin ||A p - QS||^2 subject to A[0] p = QS[0] (eq. CWENO:Popt).

        Null-space method; works for any number of right-hand sides.
        """
        nb = A.shape[1]
        Qc, Rc = np.linalg.qr(A[0].reshape(-1, 1), mode="complete")
        r = Rc[0, 0]
        q1 = Qc[:, 0]
        Z = Qc[:, 1:]
        y1 = QS[0] / r                                   # [nv]
        rhs = QS - np.outer(A @ q1, y1)
        z, _, rank, _ = np.linalg.lstsq(A @ Z, rhs, rcond=None)
        if rank < nb - 1:
            raise StencilError("rank-deficient least-squares system")
        return np.outer(q1, y1) + Z @ z                  # [nb, nv]

    def reconstruct_cell(self, i: int, Q: np.ndarray) -> dict:
        """Everything for cell i: Q is [n_vars, n_cells]."""
        d, nb = self.d, self.nb
        S0, Ss = self.stencils(i)
        extra = []
        for sec in Ss:
            if sec is not None:
                for j in sec[1:]:
                    if j not in S0 and j not in extra:
                        extra.append(j)
        allc = list(S0) + extra
        A_all = self.stencil_averages(i, allc)
        row = {j: k for k, j in enumerate(allc)}
        A = A_all[: len(S0)]
        QS = Q[:, S0].T                                   # [n_e, nv]
        popt = self.constrained_lsq(A, QS)                # [nb, nv]

        lam = self.lam.copy()
        Ps = np.zeros((d + 1, nb, Q.shape[0]))
        alive = np.ones(d + 1, dtype=bool)
        for s, sec in enumerate(Ss):
            if sec is None:
                alive[s] = False
                continue
            As = A_all[[row[j] for j in sec]][:, : d + 1]
            if np.linalg.cond(As[1:, 1:]) > SECTOR_COND_MAX:
                alive[s] = False
                continue
            Ps[s, : d + 1] = np.linalg.solve(As, Q[:, sec].T)
        lam[1:][~alive] = 0.0
        lam = lam / lam.sum()

        p0 = (popt - np.einsum("s,slv->lv", lam[1:], Ps)) / lam[0]
        polys = np.concatenate([p0[None], Ps], axis=0)    # [d+2, nb, nv]
        sig = np.einsum("slv,lm,smv->sv", polys, self.Sigma, polys)
        if self.opts.sigma0_from == "popt":
            sig[0] = np.einsum("lv,lm,mv->v", popt, self.Sigma, popt)
        if self.opts.linear_weights:
            om = np.repeat(lam[:, None], Q.shape[0], axis=1)
        else:
            wt = lam[:, None] / (sig + self.opts.eps) ** self.opts.r
            om = wt / wt.sum(axis=0, keepdims=True)
        w = np.einsum("sv,slv->lv", om, polys)
        return dict(coeffs=w.T, sigma=sig.T, omega=om.T, popt=popt.T,
                    psec=Ps.transpose(2, 0, 1), p0=p0.T, lam=lam,
                    alive=alive, stencil=S0, sectors=Ss)

    def reconstruct(self, Q: np.ndarray, cells=None) -> dict:
        """Coefficients [nv, nb, n], sigma/omega [nv, d+2, n] over ``cells``."""
        Q = np.asarray(Q, dtype=np.float64)
        idx = range(Q.shape[1]) if cells is None else cells
        idx = list(idx)
        nv = Q.shape[0]
        co = np.empty((nv, self.nb, len(idx)))
        sg = np.empty((nv, self.d + 2, len(idx)))
        om = np.empty((nv, self.d + 2, len(idx)))
        for t, i in enumerate(idx):
            r = self.reconstruct_cell(i, Q)
            co[:, :, t] = r["coeffs"]
            sg[:, :, t] = r["sigma"]
            om[:, :, t] = r["omega"]
        return dict(coeffs=co, sigma=sg, omega=om, cells=np.array(idx))

    def tables(self, cells=None):
        """Integer tables: face_nbr [n, d+1], stencil [n, n_e], sectors [n, d+1, d+1]."""
        n = self.Cells.shape[0]
        idx = list(range(n)) if cells is None else list(cells)
        st = np.empty((len(idx), self.n_e), dtype=np.int64)
        se = -np.ones((len(idx), self.d + 1, self.d + 1), dtype=np.int64)
        for t, i in enumerate(idx):
            S0, Ss = self.stencils(i)
            st[t] = S0
            for s, sec in enumerate(Ss):
                if sec is not None:
                    se[t, s] = sec
        return dict(face_nbr=self.nbr[idx], stencil=st, sectors=se)


def evaluate_polynomial(M: int, d: int, coeffs: np.ndarray, ref_pts: np.ndarray) -> np.ndarray:
    """Point values sum_l c_l psi_l(xi) at reference points: coeffs [..., nb] -> [..., q]."""
    return coeffs @ B.evaluate(M, d, ref_pts).T
