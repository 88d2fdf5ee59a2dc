"""Pins for the oracle's face adjacency and stencil selection.

* stencil sizes printed in the paper's stencil figures (Sec. 2.1: n_e = 12 for
  triangles and 30 for tetrahedra at M = 2);
* the ring rule re-derived independently: hop distances on the face graph
  from scipy's breadth-first search, cells ordered by (hop, squared
  barycentre distance, index) with numpy arithmetic;
* cone membership on hand-built triangles with known barycentric
  coordinates;
* face adjacency invariants (symmetry, shared vertices, boundary counts).
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

from oracle import CwenoOracle, Options, face_neighbours, stencil_size, StencilError
from oracle.geometry import Geometry, barycentric
from oracle.stencils import in_cone
from synthetic import kuhn_tet_mesh, tri_mesh


def test_paper_stencil_sizes():
    assert stencil_size(2, 2, 0.0) == 12      # 2-D stencil figure, M = 2
    assert stencil_size(2, 3, 0.0) == 30      # 3-D stencil figure, M = 2
    assert stencil_size(2, 2, 1.5) == 9
    assert stencil_size(3, 2, 0.0) == 20
    assert stencil_size(3, 3, 0.0) == 60


@pytest.mark.parametrize("mk", [lambda: tri_mesh(6, 0.15, 1), lambda: tri_mesh(5, 0.15, 2, periodic=False),
                                lambda: kuhn_tet_mesh(3, 0.1, 3), lambda: kuhn_tet_mesh(3, 0.1, 4, periodic=False)])
def test_face_adjacency_invariants(mk):
    m = mk()
    nbr = face_neighbours(m.cells)
    C = m.cells.astype(np.int64)
    d = m.dim
    nb_faces = 0
    for i in range(m.n_cells):
        for k in range(d + 1):
            j = nbr[i, k]
            if j < 0:
                nb_faces += 1
                continue
            face = set(C[i].tolist()) - {int(C[i, k])}
            assert face <= set(C[j].tolist())
            assert i in nbr[j].tolist()
    if m.meta["periodic"]:
        assert nb_faces == 0
    else:
        n = m.meta["n"]
        assert nb_faces == (4 * n if d == 2 else 6 * 2 * n * n)


def test_non_manifold_face_rejected():
    cells = np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]])
    with pytest.raises(StencilError):
        face_neighbours(cells)


def _numpy_centroids(m):
    X = m.vertices[m.cells.astype(np.int64)].copy()
    for a, L in enumerate(m.box):
        if L:
            dx = X[:, 1:, a] - X[:, :1, a]
            X[:, 1:, a] = X[:, :1, a] + (dx - L * np.floor(dx / L + 0.5))
    s = X[:, 0].copy()
    for k in range(1, m.dim + 1):
        s = s + X[:, k]
    return s / (m.dim + 1)


def _bruteforce_order(m, nbr, i):
    """All cells ordered by (hop distance from i, squared offset, index)."""
    n = m.n_cells
    rows, cols = np.nonzero(nbr >= 0)
    G = csr_matrix((np.ones(len(rows)), (rows, nbr[rows, cols])), shape=(n, n))
    hop = shortest_path(G, unweighted=True, indices=i)
    c = _numpy_centroids(m)
    off = c - c[i]
    for a, L in enumerate(m.box):
        if L:
            off[:, a] = off[:, a] - L * np.floor(off[:, a] / L + 0.5)
    d2 = off[:, 0] * off[:, 0]
    for a in range(1, m.dim):
        d2 = d2 + off[:, a] * off[:, a]
    return np.lexsort((np.arange(n), d2, hop))


@pytest.mark.parametrize("dim,M,factor", [(2, 2, 1.5), (2, 3, 0.0), (3, 2, 0.0)])
def test_ring_rule_matches_bruteforce(dim, M, factor):
    m = tri_mesh(12, 0.15, 7) if dim == 2 else kuhn_tet_mesh(5, 0.1, 8)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M, stencil_factor=factor))
    rng = np.random.default_rng(0)
    for i in rng.choice(m.n_cells, 25, replace=False):
        order = _bruteforce_order(m, o.nbr, int(i))
        S0, sectors = o.stencils(int(i))
        assert list(S0) == order[: o.n_e].tolist()
        geo = o.geo
        for s, sec in enumerate(sectors):
            assert sec is not None
            admitted = [j for j in order[1:] if in_cone(geo, int(i), s, int(j))]
            assert list(sec) == [int(i)] + [int(j) for j in admitted[:dim]]


def test_cone_membership_hand_built():
    X = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)]
    assert barycentric(X, (1.0, 1.0)) == [-1.0, 1.0, 1.0]
    b = barycentric(X, (-0.25, 0.5))
    assert b == [0.75, -0.25, 0.5]
    # (1,1) lies beyond the face opposite vertex 0: cone 0 only
    verts = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0], [-0.5, 0.75], [2.0, -1.0]])
    cells = np.array([[0, 1, 2], [1, 3, 2], [0, 2, 4], [0, 5, 1]])
    geo = Geometry(verts, cells, (0.0, 0.0))
    # centroid of cell 1 = (2/3, 2/3): b = (-1/3, 2/3, 2/3)
    assert [in_cone(geo, 0, s, 1) for s in range(3)] == [True, False, False]
    # cell 2 lies across the face x = 0, opposite vertex 1
    assert [in_cone(geo, 0, s, 2) for s in range(3)] == [False, True, False]
    # cell 3 lies across the face y = 0, opposite vertex 2
    assert [in_cone(geo, 0, s, 3) for s in range(3)] == [False, False, True]


def test_tetra_barycentric_known_values():
    X = [(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)]
    assert barycentric(X, (0.25, 0.25, 0.25)) == [0.25, 0.25, 0.25, 0.25]
    assert barycentric(X, (1.0, 1.0, 1.0)) == [-2.0, 1.0, 1.0, 1.0]


def test_periodic_meshes_fill_every_sector():
    for m, M in ((tri_mesh(16, 0.15, 9), 2), (kuhn_tet_mesh(5, 0.1, 10), 2)):
        o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
        T = o.tables(range(0, m.n_cells, 3))
        assert np.all(T["sectors"] >= 0)


def test_coarse_periodic_mesh_rejected():
    m = tri_mesh(4, 0.15, 14)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=3))
    with pytest.raises(StencilError):
        o.stencils(0)
