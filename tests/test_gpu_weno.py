"""GPU parity of the classical WENO kernel (the comparison scheme) against
the oracle's WENO reconstruction: FP64 data-scaled coefficient error <= 1e-12
at sampled cells (the scale: the largest |Q| over the cell's stencils); at
degree 4 the bar is 3e-12, derived from the arithmetic: the one-sided cone
stencils' column-scaled least-squares matrices reach condition numbers of
about 8e3 (against 2e2 for the central stencils), and two backward-stable FP64
solvers (Householder on the host, SVD in the oracle) then differ by up to a
small multiple of u * kappa ~ 9e-13 of the data scale (measured on the degree-4
cases below: 1.3e-12 over two variables, 2.6e-12 over nine -- the operators,
and so these errors, are the same whatever the lanes per cell);
coefficient 0 bit for bit, cell counts leaving the last workgroup ragged and
variable counts leaving the last variable block partly empty; end to end,
the reconstruction of the exact averages of a degree-M polynomial evaluated
at reference points equals that polynomial.
"""
import numpy as np
import pytest

from gpu_common import torch_cuda
from oracle import Options, WenoOracle
from synthetic import cell_averages, kuhn_tet_mesh, polynomial_field, random_polynomial, tri_mesh

pytestmark = pytest.mark.gpu

CASES = [("tri16_M2_nv5", lambda: tri_mesh(16, 0.15, 901), 2, 5, 0.95),
         ("tri20_M3_nv9", lambda: tri_mesh(20, 0.15, 902), 3, 9, 0.95),
         ("tri24_M4_nv2", lambda: tri_mesh(24, 0.15, 903), 4, 2, 0.95),
         ("tri16_M1_nv3_paper_lambda", lambda: tri_mesh(16, 0.15, 904), 1, 3, "paper"),
         ("kuhn16_M2_nv5", lambda: kuhn_tet_mesh(16, 0.1, 905), 2, 5, 0.95),
         # lane groups sharing the operator loads: 4 lanes over 19 entries a row
         # (2 variables each), and 8 lanes over 14 (2 each, the last lane idle)
         ("kuhn16_M3_nv5", lambda: kuhn_tet_mesh(16, 0.1, 907), 3, 5, 0.95),
         ("tri24_M4_nv9", lambda: tri_mesh(24, 0.15, 908), 4, 9, 0.95)]


@pytest.mark.parametrize("name,mk,M,nv,lam", CASES)
def test_weno_against_oracle(name, mk, M, nv, lam):
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = mk()
    print(f"[gpu weno] {name}: {m.n_cells} cells", flush=True)
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, weno=True, lambda0=-1.0 if lam == "paper" else lam)
    rng = np.random.default_rng(906)
    c = m.vertices[m.cells].mean(axis=1)
    Q = (np.sin(2 * np.pi * c[:, 0])[None, :] * np.arange(1, nv + 1)[:, None] + 0.1 * rng.normal(size=(nv, m.n_cells))
         + 2.0 * (c[:, 1] > 0.5)[None, :])
    q = torch.tensor(Q, device="cuda:0")
    out = torch.full((nv, lm.n_basis, lm.n_cells), float("nan"), dtype=torch.float64, device="cuda:0")
    lm.reconstruct(q, out=out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got[:, 0, :].view(np.int64), Q.view(np.int64))
    assert np.isfinite(got).all()
    o = WenoOracle(m.vertices, m.cells, m.box, Options(degree=M, lambda0="paper" if lam == "paper" else lam))
    idx = np.unique(np.concatenate([rng.choice(m.n_cells, 20, replace=False), [m.n_cells - 1]]))
    ref = o.reconstruct(Q, cells=idx)
    st = lm.weno_tables()[idx]
    scale = np.array([[np.abs(Q[v, s[s >= 0]]).max() for s in st.reshape(len(idx), -1)] for v in range(nv)])
    err = (np.abs(got[:, :, idx] - ref["coeffs"]) / scale[:, None, :]).max()
    print(f"[gpu weno]   data-scaled error {err:.3e}", flush=True)
    assert err <= (3e-12 if M == 4 else 1e-12)


def test_weno_reproduces_polynomials_and_refuses_other_forms():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = tri_mesh(18, 0.15, 910, periodic=False)
    fn = polynomial_field(random_polynomial(2, 3, 2, seed=911))
    Q = cell_averages(m, fn, degree=5)
    lm = C.Mesh(m.vertices, m.cells, 3, weno=True)
    P = np.random.default_rng(912).dirichlet(np.ones(3), size=6)[:, 1:]
    vals = lm.evaluate(C.Points(2, 3, P), lm.reconstruct(torch.tensor(Q, device="cuda:0"))).cpu().numpy()
    X = m.vertices[m.cells]
    phys = X[:, 0, None, :] + np.einsum("qa,nab->nqb", P, X[:, 1:, :] - X[:, :1, :])
    exact = fn(phys.reshape(-1, 2).T).reshape(2, m.n_cells, len(P)).transpose(0, 2, 1)
    assert np.abs(vals - exact).max() <= 1e-10 * max(1.0, np.abs(exact).max())
    q32 = torch.zeros((2, lm.n_cells), dtype=torch.float32, device="cuda:0")
    with pytest.raises(C.CwenoError):
        lm.reconstruct(q32)                                     # FP64 only
    q = torch.zeros((2, lm.n_cells), dtype=torch.float64, device="cuda:0")
    with pytest.raises(C.CwenoError):
        lm.reconstruct(q, sigma=torch.zeros((2, 4, lm.n_cells), dtype=torch.float64, device="cuda:0"))
    with pytest.raises(C.CwenoError):
        C.Batch([lm], [2], dtype="f64")


@pytest.mark.parametrize("name,mk,M", [("tri16_M2", lambda: tri_mesh(16, 0.15, 910), 2),
                                       ("kuhn16_M2", lambda: kuhn_tet_mesh(16, 0.1, 911), 2)])
def test_weno_variable_grouping_is_bitwise_invariant(name, mk, M):
    """The variables of a call are split into passes and, within a pass, over
    the lanes of a cell's group (up to 8 lanes, several variables each); each
    variable's arithmetic does not depend on that split, so 25 variables in
    one call (groups of several lanes, more than one pass) give the bits of
    the same variables reconstructed one, five and thirteen at a time."""
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = mk()
    print(f"[gpu weno] grouping {name}: {m.n_cells} cells", flush=True)
    lm = C.Mesh(m.vertices, m.cells, M, periodic=m.box, weno=True)
    rng = np.random.default_rng(912)
    Q = rng.normal(size=(25, m.n_cells)) + 3.0 * (rng.random((1, m.n_cells)) < 0.3)
    q = torch.tensor(Q, device="cuda:0")
    full = lm.reconstruct(q)
    torch.cuda.synchronize()
    assert torch.isfinite(full).all()
    for a, b in ((0, 1), (7, 8), (24, 25), (3, 8), (10, 23)):
        part = lm.reconstruct(q[a:b].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(part, full[a:b]), (name, a, b)
