"""Host builder (C ABI, CPU only) against the oracle.

* integer tables (face neighbours, central stencils, sectors) bit for bit;
* the oscillation matrix;
* per-cell operators: pinv (Q_stencil - Q_i) equals the oracle's P_opt and
  binv (Q_sector - Q_i) its sectorial polynomials;
* error paths of cweno_mesh_create;
* the shared library exports every function declared in include/cweno.h.
"""
import os
import re

import numpy as np
import pytest

import paper_1612_09335_amd as C
from oracle import CwenoOracle, Options, sigma_matrix
from synthetic import kuhn_tet_mesh, tri_mesh
from synthetic.meshes import SimplexMesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = [
    ("tri16p_M2_f1.5", lambda: tri_mesh(16, 0.15, 3), 2, 1.5, "cone"),
    ("tri12p_M3", lambda: tri_mesh(12, 0.15, 4), 3, 0.0, "cone"),
    ("tri14_M4_nonper", lambda: tri_mesh(14, 0.15, 5, periodic=False), 4, 0.0, "cone"),
    ("tri10p_M1_face", lambda: tri_mesh(10, 0.15, 6), 1, 0.0, "face"),
    ("kuhn5p_M2", lambda: kuhn_tet_mesh(5, 0.1, 7), 2, 0.0, "cone"),
    ("kuhn6p_M3", lambda: kuhn_tet_mesh(6, 0.1, 8), 3, 0.0, "cone"),
    ("kuhn4_M2_nonper", lambda: kuhn_tet_mesh(4, 0.1, 9, periodic=False), 2, 0.0, "cone"),
]


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "cweno.h")).read()
    declared = set(re.findall(r"\b(cweno_[a-z_]+)\s*\(", hdr))
    assert declared == set(C.SYMBOLS)
    for name in declared:
        assert hasattr(C.lib, name)
    assert C.lib.cweno_abi_version() == 1


@pytest.mark.parametrize("name,mk,M,factor,rule", CASES, ids=[c[0] for c in CASES])
def test_tables_and_operators_match_oracle(name, mk, M, factor, rule):
    m = mk()
    lib_mesh = C.Mesh(m.vertices, m.cells, M, periodic=m.box, stencil_factor=factor, sector_rule=rule,
                      host_only=True)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M, stencil_factor=factor, sector_rule=rule))
    T = lib_mesh.tables()
    To = o.tables()
    assert np.array_equal(T["face_nbr"], To["face_nbr"])
    assert np.array_equal(T["stencil"], To["stencil"])
    assert np.array_equal(T["sectors"], To["sectors"])
    np.testing.assert_allclose(lib_mesh.sigma_matrix(), sigma_matrix(M, m.dim)[1:, 1:], rtol=0,
                               atol=1e-13 * np.abs(sigma_matrix(M, m.dim)).max())
    rng = np.random.default_rng(17)
    Q = rng.normal(size=(3, m.n_cells)) + 5.0 * (rng.random(m.n_cells) < 0.2)
    d = m.dim
    for i in rng.choice(m.n_cells, 12, replace=False):
        i = int(i)
        r = o.reconstruct_cell(i, Q)
        P, B, _ = lib_mesh.operators(i)
        S0 = T["stencil"][i]
        scale = np.abs(Q[:, S0]).max(axis=1)
        popt = P @ (Q[:, S0[1:]] - Q[:, [i]]).T              # [nb-1, nv]
        err = np.abs(popt.T - r["popt"][:, 1:]).max(axis=1) / scale
        assert err.max() <= 1e-12, err
        for s in range(d + 1):
            sec = T["sectors"][i, s]
            if sec[0] < 0 or not r["alive"][s]:
                assert not r["alive"][s] and np.all(B[s] == 0)
                continue
            ps = B[s] @ (Q[:, sec[1:]] - Q[:, [i]]).T
            np.testing.assert_allclose(ps.T, r["psec"][:, s, 1:d + 1], rtol=0, atol=1e-12 * scale.max())


def test_dropped_sectors_counted_on_bounded_mesh():
    m = tri_mesh(8, 0.15, 11, periodic=False)
    lib_mesh = C.Mesh(m.vertices, m.cells, 2, host_only=True)
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=2))
    dropped = 0
    for i in range(m.n_cells):
        dropped += sum(s is None for s in o.stencils(i)[1])
    assert lib_mesh.n_dropped == dropped > 0


def _expect(status, fn):
    with pytest.raises(C.CwenoError) as e:
        fn()
    assert e.value.name == status


def test_error_paths():
    m = tri_mesh(8, 0.15, 12)
    V, Cc = m.vertices, m.cells
    _expect("CWENO_E_ARG", lambda: C.Mesh(V, Cc, 5, periodic=m.box, host_only=True))
    _expect("CWENO_E_ARG", lambda: C.Mesh(V, Cc, 2, periodic=m.box, lambda0=1.5, host_only=True))
    bad = Cc.copy()
    bad[3, 1] = len(V) + 7
    _expect("CWENO_E_MESH", lambda: C.Mesh(V, bad, 2, periodic=m.box, host_only=True))
    degen = Cc.copy()
    degen[5, 2] = degen[5, 1]
    _expect("CWENO_E_MESH", lambda: C.Mesh(V, degen, 2, periodic=m.box, host_only=True))
    # three triangles on one edge
    V3 = np.array([[0, 0], [1, 0], [0.5, 1], [0.5, -1], [2, 0.5]], dtype=float)
    C3 = np.array([[0, 1, 2], [0, 1, 3], [0, 1, 4]])
    _expect("CWENO_E_MESH", lambda: C.Mesh(V3, C3, 1, host_only=True))
    # too few cells to fill the central stencil
    small = tri_mesh(2, 0.1, 13, periodic=False)
    _expect("CWENO_E_STENCIL", lambda: C.Mesh(small.vertices, small.cells, 3, host_only=True))
    # periodic mesh too coarse for the stencil
    coarse = tri_mesh(4, 0.15, 14)
    _expect("CWENO_E_PERIODIC", lambda: C.Mesh(coarse.vertices, coarse.cells, 3, periodic=coarse.box,
                                               host_only=True))


def test_similarity_transform_keeps_tables_and_operators():
    m = tri_mesh(10, 0.15, 15, periodic=False)
    th = 0.4
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    V2 = 2.5 * m.vertices @ R.T + np.array([3.0, 1.0])
    a = C.Mesh(m.vertices, m.cells, 3, host_only=True)
    b = C.Mesh(V2, m.cells, 3, host_only=True)
    Ta, Tb = a.tables(), b.tables()
    assert np.array_equal(Ta["stencil"], Tb["stencil"]) and np.array_equal(Ta["sectors"], Tb["sectors"])
    for i in (0, 37, 111):
        Pa, Ba, _ = a.operators(i)
        Pb, Bb, _ = b.operators(i)
        np.testing.assert_allclose(Pb, Pa, atol=1e-11 * np.abs(Pa).max())
        np.testing.assert_allclose(Bb, Ba, atol=1e-11 * np.abs(Ba).max())


def test_renumbering_permutes_tables():
    """Renumbering cells and vertices (each cell's vertex order kept) permutes
    the central and sector stencils and the host operators, nothing else."""
    m = kuhn_tet_mesh(5, 0.1, 71)
    rng = np.random.default_rng(72)
    pc = rng.permutation(m.n_cells)
    pv = rng.permutation(m.n_vertices)
    inv_v = np.empty_like(pv)
    inv_v[pv] = np.arange(len(pv))
    a = C.Mesh(m.vertices, m.cells, 2, periodic=m.box, host_only=True)
    b = C.Mesh(m.vertices[pv], inv_v[m.cells[pc]].astype(np.int32), 2, periodic=m.box, host_only=True)
    ta, tb = a.tables(), b.tables()
    assert np.array_equal(pc[tb["stencil"]], ta["stencil"][pc])
    sb = tb["sectors"]
    assert np.array_equal(np.where(sb >= 0, pc[np.maximum(sb, 0)], -1), ta["sectors"][pc])
    for k in (0, 17, m.n_cells - 1):
        Pa, Ba, _ = a.operators(int(pc[k]))
        Pb, Bb, _ = b.operators(k)
        assert np.array_equal(Pa, Pb) and np.array_equal(Ba, Bb)
