"""GPU test of the batched reconstruction that allocates nothing
(cweno_batch_run_noalloc, called through the C ABI with ctypes; collected
last, so that its failure hides no other test).

Its launch table and work list live in a static device array: its results
must equal those of the allocating batched form (cweno_batch_create/run) and
of cweno_reconstruct bit for bit, on two calls in a row, the second with a
smaller input (fewer and smaller meshes, fewer variables) than the first;
sizes beyond the array are refused with CWENO_E_ARG.
"""
import ctypes

import numpy as np
import pytest

from gpu_common import torch_cuda
from synthetic import kuhn_tet_mesh, tri_mesh

pytestmark = pytest.mark.gpu

FIRST = [(lambda: tri_mesh(24, 0.15, 501), 3, 9), (lambda: kuhn_tet_mesh(7, 0.1, 502), 2, 5),
         (lambda: tri_mesh(16, 0.15, 503), 4, 4), (lambda: kuhn_tet_mesh(6, 0.1, 504), 3, 7),
         (lambda: tri_mesh(30, 0.15, 505), 2, 3)]
SECOND = [(lambda: tri_mesh(10, 0.15, 511), 3, 2), (lambda: kuhn_tet_mesh(4, 0.1, 512), 2, 1)]


def _noalloc(C, meshes, qs, outs, dtype):
    n = len(meshes)
    mp = (ctypes.c_void_p * n)(*[lm._h.value for lm in meshes])
    nv = (ctypes.c_int * n)(*[q.shape[0] for q in qs])
    qp = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    return C.lib.cweno_batch_run_noalloc(n, mp, nv, {"f64": C.F64, "f32": C.F32}[dtype], qp, op, None)


def _case(torch, C, spec, dtype, seed):
    tdt = {"f64": torch.float64, "f32": torch.float32}[dtype]
    raw = [(mk(), M, nv) for mk, M, nv in spec]
    meshes = [C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops=dtype) for m, M, _ in raw]
    rng = np.random.default_rng(seed)
    qs = [torch.tensor(rng.normal(size=(nv, m.n_cells)) + 3.0 * (rng.random(m.n_cells) < 0.2), dtype=tdt,
                       device="cuda:0") for m, _, nv in raw]
    return meshes, qs


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_batch_matches_allocating_forms(dtype):
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    for call, (spec, seed) in enumerate(((FIRST, 1), (SECOND, 2))):
        meshes, qs = _case(torch, C, spec, dtype, seed)
        print(f"[gpu noalloc] {dtype} call {call}: {len(meshes)} meshes, "
              f"{sum(lm.n_cells for lm in meshes)} cells", flush=True)
        outs = [torch.full((q.shape[0], lm.n_basis, lm.n_cells), float("nan"), dtype=q.dtype, device="cuda:0")
                for lm, q in zip(meshes, qs)]
        refs = [lm.reconstruct(q) for lm, q in zip(meshes, qs)]
        batch = C.Batch(meshes, [q.shape[0] for q in qs], dtype=dtype)
        bouts = [torch.full_like(r, float("nan")) for r in refs]
        batch.run(qs, bouts)
        torch.cuda.synchronize()
        assert _noalloc(C, meshes, qs, outs, dtype) == 0, C.lib.cweno_last_error().decode()
        torch.cuda.synchronize()
        for o, r, b in zip(outs, refs, bouts):
            assert torch.equal(o, b)
            assert torch.equal(o, r)
        del batch


def test_noalloc_batch_refuses_sizes_beyond_its_scratch():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = tri_mesh(10, 0.15, 521)
    lm = C.Mesh(m.vertices, m.cells, 2, periodic=m.box, ops="f64")
    q = torch.zeros((9, m.n_cells), dtype=torch.float64, device="cuda:0")
    out = torch.zeros((9, lm.n_basis, lm.n_cells), dtype=torch.float64, device="cuda:0")
    # 300 requests of one 9-variable block each: more table entries than the 256 it holds
    st = _noalloc(C, [lm] * 300, [q] * 300, [out] * 300, "f64")
    assert st == -1 and "static scratch" in C.lib.cweno_last_error().decode()
    # more than 65,536 blocks of 256 cells in all: one large mesh
    big = tri_mesh(600, 0.15, 522)
    bl = C.Mesh(big.vertices, big.cells, 1, periodic=big.box, ops="f64")
    qb = torch.zeros((1, big.n_cells), dtype=torch.float64, device="cuda:0")
    ob = torch.zeros((1, bl.n_basis, bl.n_cells), dtype=torch.float64, device="cuda:0")
    st = _noalloc(C, [bl] * 30, [qb] * 30, [ob] * 30, "f64")
    assert st == -1 and "static scratch" in C.lib.cweno_last_error().decode()
