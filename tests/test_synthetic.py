"""The input generator: mesh sizes, conformity and averaging-rule exactness."""
import itertools
import math

import numpy as np

from synthetic import kuhn_tet_mesh, tri_mesh, workload_fields
from synthetic.fields import averaging_rule


def test_rules_exact():
    for dim in (2, 3):
        for deg in (5, 7):
            lam, w = averaging_rule(dim, deg)
            assert abs(w.sum() - 1.0) < 1e-14
            for e in itertools.product(range(deg + 1), repeat=dim):
                if sum(e) > deg:
                    continue
                val = (w * np.prod(lam[:, 1:] ** np.array(e), axis=1)).sum()
                exact = math.prod(math.factorial(k) for k in e) * math.factorial(dim) / math.factorial(sum(e) + dim)
                assert abs(val - exact) < 1e-15


def test_mesh_sizes_and_volume():
    m = tri_mesh(64, 0.15, 1)
    assert m.n_cells == 8192 and m.n_vertices == 4096
    t = kuhn_tet_mesh(8, 0.1, 2)
    assert t.n_cells == 6 * 512 and t.n_vertices == 512
    # unwrapped cells tile the unit box: volumes sum to 1
    for mesh in (m, t):
        X = mesh.vertices[mesh.cells.astype(np.int64)]
        dx = X[:, 1:] - X[:, :1]
        dx = dx - np.round(dx)
        vol = np.abs(np.linalg.det(dx)) / math.factorial(mesh.dim)
        assert abs(vol.sum() - 1.0) < 1e-12 and vol.min() > 0


def test_fields_deterministic_and_finite():
    m = tri_mesh(16, 0.15, 3)
    a = workload_fields(m, "mhd2d", 7)
    b = workload_fields(m, "mhd2d", 7)
    assert a.shape == (9, m.n_cells) and np.array_equal(a, b) and np.isfinite(a).all()
    assert a[0].min() > 0
