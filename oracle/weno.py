"""Classical unstructured WENO reconstruction -- oracle side (TEST INFRASTRUCTURE).

The reconstruction the paper compares CWENO with (Sec. 4, efficiency
discussion): n_s = 1 + 2(d+1) stencils -- one central, d+1 forward sector
and d+1 reverse sector stencils -- each of n_e cells and each producing a
polynomial of degree M, combined with nonlinear weights.  The paper gives
only this outline; the readings taken here:

* central stencil: the CWENO central stencil (same fill);
* forward sector s: the fill restricted to barycentres in the open cone at
  vertex s spanned by the edges to the other vertices (the CWENO sector
  cone), filled to n_e cells; reverse sector s: the opposite cone at vertex
  s (every barycentric coordinate but the s-th below -1e-12), filled to n_e;
* each polynomial: the constrained least squares of eq. CWENO:Popt on its
  own stencil (its cell average matched exactly);
* indicators sigma_j = p_j^T Sigma p_j with the universal Sigma of Sec. 2.1;
* linear weights: lambda_0 for the central stencil (default 0.95; 'paper':
  1e5 against 1 per sector stencil, normalised), the rest (1 - lambda_0) /
  (2(d+1)) each; a stencil that cannot be filled is dropped and the others
  renormalised;
* omega~_j = lambda_j / (sigma_j + eps)^r, omega = omega~ / sum omega~,
  w = sum_j omega_j P_j (eqs. weights, weights2 with all polynomials of
  degree M).
"""
from __future__ import annotations

import numpy as np

from .cweno import CwenoOracle, Options
from .stencils import weno_stencils


class WenoOracle:
    """Plain FP64 classical WENO reconstruction of one mesh."""

    def __init__(self, vertices, cells, box, opts: Options, nbr=None):
        self.cw = CwenoOracle(vertices, cells, box, opts, nbr=nbr)
        self.d, self.M, self.nb, self.n_e = self.cw.d, self.cw.M, self.cw.nb, self.cw.n_e
        self.n_s = 1 + 2 * (self.d + 1)
        if opts.lambda0 == "paper":       # 1e5 for the central stencil, 1 per sector stencil, normalised
            tot = 1e5 + (self.n_s - 1)
            self.lam = np.array([1e5 / tot] + [1.0 / tot] * (self.n_s - 1))
        else:
            l0 = 0.95 if opts.lambda0 == 0.0 else float(opts.lambda0)
            self.lam = np.array([l0] + [(1.0 - l0) / (self.n_s - 1)] * (self.n_s - 1))
        self.opts = opts
        self._cache = {}

    def stencils(self, i: int):
        """[central, forward_0 .. forward_d, reverse_0 .. reverse_d]; None = unfillable."""
        c = self._cache.get(i)
        if c is None:
            S0, _ = self.cw.stencils(i)
            c = [S0] + weno_stencils(self.cw.geo, self.cw.nbr, i, self.n_e)
            self._cache[i] = c
        return c

    def reconstruct_cell(self, i: int, Q: np.ndarray) -> dict:
        nv = Q.shape[0]
        polys = np.zeros((self.n_s, self.nb, nv))
        alive = np.zeros(self.n_s, dtype=bool)
        for j, S in enumerate(self.stencils(i)):
            if S is None:
                continue
            A = self.cw.stencil_averages(i, S)
            polys[j] = CwenoOracle.constrained_lsq(A, Q[:, S].T)
            alive[j] = True
        lam = np.where(alive, self.lam, 0.0)
        lam = lam / lam.sum()
        sig = np.einsum("slv,lm,smv->sv", polys, self.cw.Sigma, polys)
        wt = lam[:, None] / (sig + self.opts.eps) ** self.opts.r
        om = wt / wt.sum(axis=0, keepdims=True)
        w = np.einsum("sv,slv->lv", om, polys)
        return dict(coeffs=w.T, sigma=sig.T, omega=om.T, polys=polys, lam=lam, alive=alive)

    def reconstruct(self, Q: np.ndarray, cells=None) -> dict:
        Q = np.asarray(Q, dtype=np.float64)
        idx = list(range(Q.shape[1]) if cells is None else cells)
        nv = Q.shape[0]
        co = np.empty((nv, self.nb, len(idx)))
        sg = np.empty((nv, self.n_s, len(idx)))
        om = np.empty((nv, self.n_s, len(idx)))
        for t, i in enumerate(idx):
            r = self.reconstruct_cell(i, Q)
            co[:, :, t], sg[:, :, t], om[:, :, t] = r["coeffs"], r["sigma"], r["omega"]
        return dict(coeffs=co, sigma=sg, omega=om, cells=np.array(idx))

    def tables(self, cells=None):
        """Stencils [n, n_s, n_e] with -1 rows for unfillable stencils."""
        n = self.cw.Cells.shape[0]
        idx = list(range(n)) if cells is None else list(cells)
        out = -np.ones((len(idx), self.n_s, self.n_e), dtype=np.int64)
        for t, i in enumerate(idx):
            for j, S in enumerate(self.stencils(i)):
                if S is not None:
                    out[t, j] = S
        return out
