"""Exact pins of the oracle's rules that the paper leaves open, and of its
options (Sec. 2.1; the readings are listed in the oracle's module headers).

* Dropped sectors.  The paper assumes every sectorial stencil exists and is
  non-degenerate.  The reading: a sector is dropped when its cone holds too
  few cells or when its d x d system (eq. CWENO:Ps, orthonormal linear basis)
  has 2-norm condition number above 1e10; lambda_s := 0 and the remaining
  linear weights are renormalised.  Pinned here by
  - the emptiness decision re-derived on every cell of bounded dyadic meshes
    from exact barycentric coordinates and breadth-first hop distances on a
    brute-force face graph;
  - the whole exact-rational pipeline (its own sector decisions, its own
    renormalisation in rationals) on boundary cells that lose sectors;
  - a hand-built sector with exactly collinear barycentres, and a sweep of
    perturbations across the 1e10 threshold decided exactly from the
    characteristic polynomial of B^T B.
* ``sector_rule='face'``: hand-built four-triangle mesh with known
  neighbours, and the exact pipeline with sectors from a brute-force
  adjacency.
* ``sigma0_from='popt'``: the exact pipeline with sigma_0 of P_opt.
* Classical WENO with the paper's linear weights (1e5 central, 1 per sector
  stencil, normalised over the stencils that exist): exact per-stencil KKT
  solves, indicators and weights.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

from exact_rational import ExactCell, cond_exceeds, exact_cweno, exact_weno, lin_unnormalised, point_values
from oracle import CwenoOracle, Options, WenoOracle, evaluate_polynomial
from oracle.geometry import Geometry
from oracle.stencils import CONE_TOL, MAX_RINGS, sector_stencils
from synthetic import kuhn_tet_mesh, tri_mesh


def _bounded(kind):
    if kind == "tri":
        return tri_mesh(8, 0.15, 41, periodic=False, dyadic=16)
    return kuhn_tet_mesh(3, 0.1, 42, periodic=False, dyadic=16)


def _brute_adjacency(cells):
    """nbr[i][k]: the other cell holding every vertex of cell i but local
    vertex k (searched over all cells), or -1."""
    C = [set(map(int, c)) for c in cells]
    n, nv = len(C), len(cells[0])
    out = -np.ones((n, nv), dtype=np.int64)
    for i in range(n):
        for k in range(nv):
            face = C[i] - {int(cells[i][k])}
            hits = [j for j in range(n) if j != i and face <= C[j]]
            assert len(hits) <= 1
            if hits:
                out[i, k] = hits[0]
    return out


def _exact_bary(X, p):
    """Barycentric coordinates of p in the simplex X, exact rationals."""
    d = len(p)
    A = [[X[k][a] for k in range(d + 1)] for a in range(d)] + [[Fr(1)] * (d + 1)]
    # Gauss-Jordan on the (d+1) x (d+1) system
    M = [row[:] + [rhs] for row, rhs in zip(A, list(p) + [Fr(1)])]
    for c in range(d + 1):
        piv = next(r for r in range(c, d + 1) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        M[c] = [x / M[c][c] for x in M[c]]
        for r in range(d + 1):
            if r != c and M[r][c] != 0:
                M[r] = [x - M[r][c] * y for x, y in zip(M[r], M[c])]
    return [M[r][d + 1] for r in range(d + 1)]


@pytest.mark.parametrize("kind", ["tri", "tet"])
def test_unfillable_sector_decision_bruteforce(kind):
    """A cone sector is unfillable exactly when fewer than d cells within the
    ring limit have barycentres strictly inside the open cone; a filled
    sector takes admitted cells of the nearest rings only."""
    m = _bounded(kind)
    d = m.dim
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=1))
    nbr = _brute_adjacency(m.cells)
    assert np.array_equal(nbr, o.nbr)
    n = m.n_cells
    rows, cols = np.nonzero(nbr >= 0)
    hop_all = shortest_path(csr_matrix((np.ones(len(rows)), (rows, nbr[rows, cols])), shape=(n, n)),
                            unweighted=True)
    X = [[[Fr(float(x)) for x in m.vertices[v]] for v in c] for c in m.cells]
    cent = [[sum((x[a] for x in Xc), Fr(0)) / (d + 1) for a in range(d)] for Xc in X]
    tol = Fr(CONE_TOL)
    n_dropped = 0
    for i in range(n):
        _, secs = o.stencils(i)
        hop = hop_all[i]
        bary = {j: _exact_bary(X[i], cent[j]) for j in range(n) if j != i and hop[j] <= MAX_RINGS}
        for s in range(d + 1):
            adm = [j for j, b in bary.items() if all(b[t] > tol for t in range(d + 1) if t != s)]
            if len(adm) < d:
                assert secs[s] is None, (i, s)
                n_dropped += 1
                continue
            sec = secs[s]
            assert sec is not None and sec[0] == i and len(sec) == d + 1, (i, s)
            assert set(sec[1:]) <= set(adm)
            unchosen = [hop[j] for j in adm if j not in sec]
            if unchosen:
                assert max(hop[j] for j in sec[1:]) <= min(unchosen)
    assert n_dropped > 0


def _dyadic_data(m, seed):
    rng = np.random.default_rng(seed)
    base = rng.integers(-64, 64, size=m.n_cells) / 16.0
    c = m.vertices[m.cells.astype(np.int64)].mean(axis=1)
    return np.stack([base, base + 8.0 * (c[:, 0] > 0.45), np.full(m.n_cells, 0.75)])


def _ref_pts(d):
    return np.array([[0.0] * d, [0.25] * d, [0.5] + [0.125] * (d - 1), [0.1] * d])


def _compare(o, r, ex, Q, v, i, M, d):
    pts = _ref_pts(d)
    got = evaluate_polynomial(M, d, r["coeffs"][v], pts)
    scale = max(1.0, np.abs(Q[v, o.stencils(i)[0]]).max())
    np.testing.assert_allclose(got, point_values(ex["cell"], ex["w"], pts), rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(r["sigma"][v], [float(s) for s in ex["sigma"]], rtol=1e-10, atol=1e-22 * scale ** 2)
    np.testing.assert_allclose(r["omega"][v], [float(x) for x in ex["omega"]], rtol=0, atol=1e-12)


def _lam(d):
    return [Fr(95, 100)] + [Fr(5, 100 * (d + 1))] * (d + 1)


@pytest.mark.parametrize("kind,M", [("tri", 2), ("tri", 3), ("tet", 2)])
def test_dropped_sectors_exact_pipeline(kind, M):
    """Boundary cells losing one or more sectors: the exact pipeline decides
    the drops itself and renormalises lambda in rationals."""
    m = _bounded(kind)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    Q = _dyadic_data(m, 43)
    picked = []
    for i in range(m.n_cells):
        try:
            secs = o.stencils(i)[1]
        except Exception:
            continue
        k = sum(s is None for s in secs)
        if k and (not picked or k not in [p[1] for p in picked]):
            picked.append((i, k))
        if len(picked) == 2:
            break
    assert picked
    for i, k in picked:
        r = o.reconstruct_cell(i, Q)
        assert int((~r["alive"]).sum()) == k
        for v in range(Q.shape[0]):
            ex = exact_cweno(o, i, Q[v].tolist(), _lam(m.dim))
            assert list(ex["alive"]) == list(r["alive"])
            lam_exp = [float(x) for x in ex["lam"]]
            np.testing.assert_allclose(r["lam"], lam_exp, rtol=4e-15, atol=0)
            # a dropped sector carries no weight at all
            assert all(r["omega"][v][s + 1] == 0.0 for s in range(m.dim + 1) if not r["alive"][s])
            _compare(o, r, ex, Q, v, i, M, m.dim)


def _collinear_case(delta):
    """Regular bounded 8x8 triangulation; the first triangle of each square of
    row 3 has its barycentre on y = (3 + 1/3) h.  Sector 0 of the cell in
    square 3 is set to (that cell, the cell in square 5, the cell in square
    7): collinear barycentres.  ``delta`` lifts the top vertex of square 7's
    triangle, moving its barycentre off the line by delta / 3."""
    m = tri_mesh(8, 0.0, 44, periodic=False)
    i0, j, k = 2 * (8 * 3 + 3), 2 * (8 * 3 + 5), 2 * (8 * 3 + 7)
    V = m.vertices.copy()
    top = [int(v) for v in m.cells[k] if V[v, 1] > 3.5 / 8]
    assert len(top) == 1
    V[top[0], 1] += delta
    return m, V, i0, [i0, j, k]


def _fixed_tables(m, V, M, i0, sec0):
    base = CwenoOracle(V, m.cells, m.box, Options(degree=M))
    T = base.tables()
    T["sectors"][i0, 0] = sec0
    return T


def test_collinear_sector_dropped_exact():
    m, V, i0, sec0 = _collinear_case(0.0)
    M = 2
    T = _fixed_tables(m, V, M, i0, sec0)
    o = CwenoOracle(V, m.cells, m.box, Options(degree=M), stencils=(T["stencil"], T["sectors"]))
    ec = ExactCell(o, i0)
    L = [lin_unnormalised(2, ec.barycentre_ref(c)) for c in sec0[1:]]
    assert cond_exceeds(L, 2)                                # exactly singular
    Q = _dyadic_data(m, 45)
    r = o.reconstruct_cell(i0, Q)
    assert not r["alive"][0] and r["alive"][1:].all()
    for v in range(Q.shape[0]):
        ex = exact_cweno(o, i0, Q[v].tolist(), _lam(2))
        assert ex["alive"] == [False, True, True]
        _compare(o, r, ex, Q, v, i0, M, 2)


def test_condition_threshold_exact():
    """Perturbations of the collinear sector across cond = 1e10: the oracle
    keeps the sector exactly when the exact condition number is at most
    1e10 (decisions within 1% of the threshold are not asserted)."""
    seen = set()
    for e in range(24, 46):
        delta = 2.0 ** -e
        m, V, i0, sec0 = _collinear_case(delta)
        T = _fixed_tables(m, V, 1, i0, sec0)
        o = CwenoOracle(V, m.cells, m.box, Options(degree=1), stencils=(T["stencil"], T["sectors"]))
        ec = ExactCell(o, i0)
        L = [lin_unnormalised(2, ec.barycentre_ref(c)) for c in sec0[1:]]
        hi, lo = cond_exceeds(L, 2, 1.01e10), cond_exceeds(L, 2, 0.99e10)
        if hi != lo:
            continue
        Q = _dyadic_data(m, 46)
        alive = bool(o.reconstruct_cell(i0, Q)["alive"][0])
        assert alive == (not hi), (e, alive)
        seen.add(alive)
    assert seen == {True, False}


def test_face_rule_hand_built():
    """Sector s of the face rule: the cell and its face neighbours except the
    one across the face opposite vertex s; a missing neighbour empties it."""
    verts = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0], [-0.5, 0.75], [2.0, -1.0]])
    cells = np.array([[0, 1, 2], [1, 3, 2], [0, 2, 4], [0, 5, 1]])
    geo = Geometry(verts, cells, (0.0, 0.0))
    nbr = _brute_adjacency(cells)
    # cell 0: across {1,2} (opposite vertex 0) is cell 1, across {0,2} cell 2, across {0,1} cell 3
    assert nbr[0].tolist() == [1, 2, 3]
    assert sector_stencils(geo, nbr, 0, "face") == [[0, 2, 3], [0, 1, 3], [0, 1, 2]]
    for c in (1, 2, 3):
        assert sector_stencils(geo, nbr, c, "face") == [None, None, None]


@pytest.mark.parametrize("kind,M", [("tri", 2), ("tet", 2)])
def test_face_rule_exact_pipeline(kind, M):
    m = _bounded(kind)
    d = m.dim
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M, sector_rule="face"))
    nbr = _brute_adjacency(m.cells)
    Q = _dyadic_data(m, 47)
    rng = np.random.default_rng(48)
    cand = [i for i in range(m.n_cells) if (nbr[i] >= 0).all()]
    bnd = [i for i in range(m.n_cells) if (nbr[i] < 0).sum() == 1]
    for i in [int(x) for x in rng.choice(cand, 2, replace=False)] + bnd[:1]:
        secs = [None if any(nbr[i, t] < 0 for t in range(d + 1) if t != s)
                else [i] + [int(nbr[i, t]) for t in range(d + 1) if t != s] for s in range(d + 1)]
        assert o.stencils(i)[1] == secs
        r = o.reconstruct_cell(i, Q)
        for v in range(Q.shape[0]):
            ex = exact_cweno(o, i, Q[v].tolist(), _lam(d), sectors=secs)
            assert list(ex["alive"]) == list(r["alive"])
            _compare(o, r, ex, Q, v, i, M, d)


@pytest.mark.parametrize("kind,M", [("tri", 2), ("tri", 3), ("tet", 2)])
def test_sigma0_from_popt_exact(kind, M):
    m = _bounded(kind)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M, sigma0_from="popt"))
    o_p0 = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    Q = _dyadic_data(m, 49)
    n = m.n_cells
    for i in (n // 2 + 3, n // 3):
        r = o.reconstruct_cell(i, Q)
        r0 = o_p0.reconstruct_cell(i, Q)
        for v in range(2):
            ex = exact_cweno(o, i, Q[v].tolist(), _lam(m.dim), sigma0_popt=True)
            _compare(o, r, ex, Q, v, i, M, m.dim)
            # on jump data sigma(P_opt) and sigma(P0) differ: the option matters
            assert abs(r["sigma"][v][0] - r0["sigma"][v][0]) > 1e-6 * abs(r0["sigma"][v][0])


@pytest.mark.parametrize("lambda0", ["paper", 0.95])
def test_weno_weights_exact(lambda0):
    """Classical WENO on a bounded dyadic mesh, interior and boundary cells
    (reverse stencils lost at the boundary are dropped and the weights
    renormalised), against exact per-stencil KKT solves."""
    m = tri_mesh(16, 0.15, 50, periodic=False, dyadic=16)
    M, d = 2, 2
    o = WenoOracle(m.vertices, m.cells, m.box, Options(degree=M, lambda0=lambda0))
    ns = o.n_s
    lam_raw = ([Fr(10 ** 5)] + [Fr(1)] * (ns - 1) if lambda0 == "paper"
               else [Fr(95, 100)] + [Fr(5, 100 * (ns - 1))] * (ns - 1))
    Q = _dyadic_data(m, 51)
    pts = _ref_pts(d)
    first = {}
    for i in range(m.n_cells):
        first.setdefault(sum(S is None for S in o.stencils(i)), i)
    assert 0 in first and max(first) >= 3
    cells = [first[0], first[2], first[max(first)]]
    for i in cells:
        r = o.reconstruct_cell(i, Q)
        for v in range(2):
            ex = exact_weno(o, i, Q[v].tolist(), lam_raw)
            np.testing.assert_allclose(r["lam"], [float(x) for x in ex["lam"]], rtol=1e-14, atol=0)
            got = evaluate_polynomial(M, d, r["coeffs"][v], pts)
            scale = max(1.0, np.abs(Q[v]).max())
            np.testing.assert_allclose(got, point_values(ex["cell"], ex["w"], pts), rtol=0, atol=1e-12 * scale)
            np.testing.assert_allclose(r["omega"][v], [float(x) for x in ex["omega"]], rtol=0, atol=1e-12)
            np.testing.assert_allclose(r["sigma"][v], [float(s) for s in ex["sigma"]], rtol=1e-10,
                                       atol=1e-22 * scale ** 2)
