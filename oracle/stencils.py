"""Face adjacency and stencil selection -- oracle side.

* Neumann (face) neighbours, Sec. 2.4: face k of cell i is its vertex set
  without local vertex k; two cells sharing that vertex set are neighbours
  across it.  A face claimed by more than two cells is an error; an unmatched
  face is a boundary face (neighbour -1).
* Central stencil S_i^0, Sec. 2.1 (eq. stencil): n_e cells, the cell itself
  first, filled by repeatedly adding neighbours of cells already reached.
* Sectorial stencils S_i^s, Sec. 2.1: d+1 cells each, the cell itself first,
  the same fill restricted to cells whose barycentre lies in the open cone
  with apex at vertex s spanned by the edges towards the other vertices (the
  cone "defined by vertex s and the opposite face").

The paper leaves the order of the recursive fill open.  Reading adopted here
(identical in the library's builder): breadth-first rings over face
neighbours; ring r is every not-yet-visited face neighbour of ring r-1,
sorted by squared barycentre distance to cell i (minimum image), ties by the
lower cell index; cells are taken ring by ring in that order until the target
count is reached.  Expansion goes through every cell of a ring, admitted or
not.  A cell is in cone s when its barycentric coordinates w.r.t. T_i satisfy
b_m > 1e-12 for every m != s.

A second sector rule (option ``sector_rule='face'``): sector s is the cell
and its face neighbours except the one across the face opposite vertex s.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, barycentric

CONE_TOL = 1e-12
MAX_RINGS = 16
# A stencil cell farther than this fraction of the period from cell i (along
# a periodic axis) makes the minimum-image reading unsafe: the mesh is too
# coarse for the stencil.
PERIODIC_REACH = 0.375


class StencilError(RuntimeError):
    pass


def face_neighbours(cells: np.ndarray) -> np.ndarray:
    """nbr[i, k] = cell across the face opposite local vertex k, or -1."""
    C = np.asarray(cells, dtype=np.int64)
    n, nv = C.shape
    owner = {}
    nbr = -np.ones((n, nv), dtype=np.int64)
    for i in range(n):
        row = C[i].tolist()
        for k in range(nv):
            key = tuple(sorted(row[:k] + row[k + 1:]))
            prev = owner.get(key)
            if prev is None:
                owner[key] = (i, k)
            elif prev == "full":
                raise StencilError(f"face {key} shared by more than two cells")
            else:
                j, kj = prev
                nbr[i, k] = j
                nbr[j, kj] = i
                owner[key] = "full"
    return nbr


def _check_reach(geo: Geometry, i: int, j: int):
    o = geo.offset(i, j)
    for a, L in enumerate(geo.box):
        if L and abs(o[a]) > PERIODIC_REACH * L:
            raise StencilError(f"stencil of cell {i} reaches too far across the periodic box")


def ring_fill(geo: Geometry, nbr: np.ndarray, i: int, n_target: int, admit=None):
    """Breadth-first ring fill; returns the selected cell list or None."""
    sel = [i]
    if n_target <= 1:
        return sel
    visited = {i}
    frontier = [i]
    for _ in range(MAX_RINGS):
        cand = set()
        for f in frontier:
            for j in nbr[f].tolist():
                if j >= 0 and j not in visited:
                    cand.add(j)
        if not cand:
            return None
        ring = sorted(cand, key=lambda j: (geo.dist2(i, j), j))
        visited.update(ring)
        for j in ring:
            if admit is None or admit(j):
                sel.append(j)
                if len(sel) == n_target:
                    return sel
        frontier = ring
    return None


def central_stencil(geo: Geometry, nbr: np.ndarray, i: int, n_e: int):
    sel = ring_fill(geo, nbr, i, n_e)
    if sel is None:
        raise StencilError(f"cannot fill the central stencil of cell {i}")
    for j in sel[1:]:
        _check_reach(geo, i, j)
    return sel


def in_cone(geo: Geometry, i: int, s: int, j: int) -> bool:
    X = geo.cell_vertices(i)
    ci = geo.centroid(i)
    o = geo.offset(i, j)
    p = tuple(ci[a] + o[a] for a in range(geo.d))
    b = barycentric(X, p)
    return all(b[m] > CONE_TOL for m in range(geo.d + 1) if m != s)


def in_reverse_cone(geo: Geometry, i: int, s: int, j: int) -> bool:
    """The cone opposite to cone s at vertex s (apex X_s, spanned by the edges
    pointing away from the other vertices): b_m < -1e-12 for every m != s."""
    X = geo.cell_vertices(i)
    ci = geo.centroid(i)
    o = geo.offset(i, j)
    p = tuple(ci[a] + o[a] for a in range(geo.d))
    b = barycentric(X, p)
    return all(b[m] < -CONE_TOL for m in range(geo.d + 1) if m != s)


def weno_stencils(geo: Geometry, nbr: np.ndarray, i: int, n_e: int):
    """The d+1 forward and d+1 reverse sector stencils of the classical
    unstructured WENO reconstruction, n_e cells each (i first), filled by the
    same ring procedure restricted to cone s or to its reverse; None when a
    stencil cannot be filled."""
    d = geo.d
    out = []
    for pred in (in_cone, in_reverse_cone):
        for s in range(d + 1):
            sel = ring_fill(geo, nbr, i, n_e, admit=lambda j, s=s, pred=pred: pred(geo, i, s, j))
            if sel is not None:
                for j in sel[1:]:
                    _check_reach(geo, i, j)
            out.append(sel)
    return out


def sector_stencils(geo: Geometry, nbr: np.ndarray, i: int, rule: str = "cone"):
    """List of d+1 sectors; each is a list of d+1 cells (i first) or None (unfillable)."""
    d = geo.d
    out = []
    for s in range(d + 1):
        if rule == "cone":
            sel = ring_fill(geo, nbr, i, d + 1, admit=lambda j, s=s: in_cone(geo, i, s, j))
        elif rule == "face":
            cand = [int(nbr[i, k]) for k in range(d + 1) if k != s]
            sel = None if any(c < 0 for c in cand) else [i] + cand
        else:
            raise ValueError(f"unknown sector rule {rule!r}")
        if sel is not None:
            for j in sel[1:]:
                _check_reach(geo, i, j)
        out.append(sel)
    return out
