"""Seeded jittered simplex meshes of the unit square / unit cube.

Two families, both conforming and (optionally) periodic:

* ``tri_mesh(n)``: an n x n grid of squares, each split into two triangles
  along a diagonal drawn at random (seeded), with every vertex jittered
  uniformly by +-``jitter``*h per coordinate (h = 1/n).  2 n^2 triangles.
* ``kuhn_tet_mesh(n)``: an n^3 grid of cubes, each split into the six Kuhn
  tetrahedra (one per permutation of the axes; every cube uses the same
  split, so the mesh is conforming across faces and across the periodic
  wrap), vertices jittered by +-``jitter``*h.  6 n^3 tetrahedra.

Periodic meshes store each vertex once (n^d vertices); a cell that straddles
the wrap simply references vertices on the other side, and consumers unwrap
by the minimum-image convention.  Non-periodic meshes have (n+1)^d vertices
and keep boundary vertices on the boundary (jitter only along the boundary).

Cell order is the natural grid order (squares / cubes row-major, their
simplices consecutive), which is the locality order a mesh generator or a
space-filling-curve renumbering would produce.  The vertex order of each cell
is the order given here; it fixes each cell's reference frame (the affine map
of Sec. 2, eq. xietaTransf, puts the first vertex at the origin).

With ``dyadic=q`` the jitter is rounded to multiples of h/q; for n a power of
two every coordinate is then a dyadic rational, exactly representable, so an
exact-rational brute-force computation can consume the mesh verbatim.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class SimplexMesh:
    """A conforming simplex mesh: vertices, cells, periodic box.

    ``box[a]`` is the period along axis ``a`` (0 = not periodic).
    """
    dim: int
    vertices: np.ndarray          # float64 [n_vertices, dim]
    cells: np.ndarray             # int32   [n_cells, dim + 1]
    box: tuple                    # period per axis, 0.0 = none
    h: float                      # nominal spacing
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(self.vertices.shape[0])


def _jitter(rng, shape, amp, h, dyadic):
    j = rng.uniform(-amp, amp, size=shape) * h
    if dyadic:
        step = h / dyadic
        j = np.round(j / step) * step
    return j


def tri_mesh(n: int, jitter: float = 0.15, seed: int = 0, periodic: bool = True,
             dyadic: int | None = None) -> SimplexMesh:
    """Jittered 2-D triangulation of the unit square with 2 n^2 triangles."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    nv1 = n if periodic else n + 1
    ii, jj = np.meshgrid(np.arange(nv1), np.arange(nv1), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()            # vertex id = j * nv1 + i
    base = np.stack([ii * h, jj * h], axis=1).astype(np.float64)
    jit = _jitter(rng, base.shape, jitter, h, dyadic)
    if not periodic:
        jit[(ii == 0) | (ii == n), 0] = 0.0
        jit[(jj == 0) | (jj == n), 1] = 0.0
    verts = base + jit
    diag = rng.integers(0, 2, size=(n, n))   # [j, i]

    def vid(i, j):
        if periodic:
            return (j % n) * n + (i % n)
        return j * (n + 1) + i

    cells = np.empty((2 * n * n, 3), dtype=np.int64)
    c = 0
    for j in range(n):
        for i in range(n):
            a, b, cc, e = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            if diag[j, i] == 0:
                cells[c] = (a, b, cc)
                cells[c + 1] = (a, cc, e)
            else:
                cells[c] = (a, b, e)
                cells[c + 1] = (b, cc, e)
            c += 2
    box = (1.0, 1.0) if periodic else (0.0, 0.0)
    return SimplexMesh(2, verts, cells.astype(np.int32), box, h,
                       name=f"tri{n}{'p' if periodic else ''}",
                       meta=dict(n=n, jitter=jitter, seed=seed, periodic=periodic))


# Kuhn split of the unit cube: for each axis permutation the path
# (0,0,0) -> +e_p0 -> +e_p1 -> (1,1,1) spans one tetrahedron.
_KUHN = []
for _perm in itertools.permutations(range(3)):
    _p = [np.zeros(3, dtype=np.int64)]
    for _ax in _perm:
        _q = _p[-1].copy()
        _q[_ax] += 1
        _p.append(_q)
    _KUHN.append(np.array(_p))


def kuhn_tet_mesh(n: int, jitter: float = 0.1, seed: int = 0, periodic: bool = True,
                  dyadic: int | None = None) -> SimplexMesh:
    """Jittered 3-D Kuhn tetrahedrisation of the unit cube, 6 n^3 tetrahedra."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    nv1 = n if periodic else n + 1
    kk, jj, ii = np.meshgrid(np.arange(nv1), np.arange(nv1), np.arange(nv1), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()   # vertex id = (k*nv1 + j)*nv1 + i
    base = np.stack([ii * h, jj * h, kk * h], axis=1).astype(np.float64)
    jit = _jitter(rng, base.shape, jitter, h, dyadic)
    if not periodic:
        for a, idx in enumerate((ii, jj, kk)):
            jit[(idx == 0) | (idx == n), a] = 0.0
    verts = base + jit

    # Vectorised over cubes: cube (i,j,k) corner offsets -> vertex ids.
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    # cube order: k outer, then j, then i (row-major in (k, j, i))
    ci = np.transpose(ci, (2, 1, 0)).ravel()
    cj = np.transpose(cj, (2, 1, 0)).ravel()
    ck = np.transpose(ck, (2, 1, 0)).ravel()
    ncube = n ** 3
    cells = np.empty((ncube, 6, 4), dtype=np.int64)
    for t, path in enumerate(_KUHN):
        for v in range(4):
            oi = ci + path[v, 0]
            oj = cj + path[v, 1]
            ok = ck + path[v, 2]
            if periodic:
                oi, oj, ok = oi % n, oj % n, ok % n
            cells[:, t, v] = (ok * nv1 + oj) * nv1 + oi
    cells = cells.reshape(ncube * 6, 4)
    box = (1.0, 1.0, 1.0) if periodic else (0.0, 0.0, 0.0)
    return SimplexMesh(3, verts, cells.astype(np.int32), box, h,
                       name=f"kuhn{n}{'p' if periodic else ''}",
                       meta=dict(n=n, jitter=jitter, seed=seed, periodic=periodic))


def workload_mesh(dim: int, n_cells_target: int, seed: int, periodic: bool = True) -> SimplexMesh:
    """Grid mesh of the given dimension whose cell count is close to a target.

    2-D: n = round(sqrt(target/2)); 3-D: n = round(cbrt(target/6)); n >= 3 so
    that a periodic stencil never wraps onto itself at the smallest sizes.
    """
    if dim == 2:
        n = max(3, int(round((n_cells_target / 2.0) ** 0.5)))
        return tri_mesh(n, 0.15, seed, periodic)
    if dim == 3:
        n = max(3, int(round((n_cells_target / 6.0) ** (1.0 / 3.0))))
        return kuhn_tet_mesh(n, 0.1, seed, periodic)
    raise ValueError("dim must be 2 or 3")


def batch_spec(n_meshes: int = 64, lo: float = 1e3, hi: float = 3e5, seed: int = 16120937):
    """Seeded recipe of a batch of uneven meshes: [(dim, n_cells_target, degree, mesh_seed)].

    Cell counts log-uniform on [lo, hi], dimension uniform in {2, 3}, degree
    uniform in {2, 3, 4}.
    """
    rng = np.random.default_rng(seed)
    out = []
    for t in range(n_meshes):
        n = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        d = int(rng.integers(2, 4))
        M = int(rng.integers(2, 5))
        out.append((d, int(round(n)), M, seed + 1 + t))
    return out


def moved_vertices(mesh: SimplexMesh, amplitude: float = 0.3, phase: float = 0.0) -> np.ndarray:
    """Vertex positions of ``mesh`` after a smooth periodic motion.

    Each axis is sheared by a sine of the next axis (cyclically):
    x_a += amplitude / (2 pi) * sin(2 pi (x_{a+1} + phase)), so the motion
    is periodic on the unit box, its gradient is at most ``amplitude`` and
    the Jacobian stays invertible (1 - amplitude^2 > 0 in 2-D,
    1 - amplitude^3 > 0 in 3-D).  The connectivity is unchanged.
    """
    V = np.asarray(mesh.vertices, dtype=np.float64)
    d = V.shape[1]
    out = V.copy()
    for a in range(d):
        out[:, a] += amplitude / (2 * np.pi) * np.sin(2 * np.pi * (V[:, (a + 1) % d] + phase))
    return out
