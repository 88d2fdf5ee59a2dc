"""Per-cell operators assembled on the GPU (CWENO_FLAG_DEVICE_OPERATORS).

The device builds the same operators as the host builder from the same
stencils (FP64 averages, Householder least squares, sector inverses); the
two differ only by rounding.  Checked: reconstructions from device-built
operators match those from host-built ones to 1e-13 of the data scale (FP64)
and the oracle to the FP64 bar; FP32 operators to the FP32 bar; the dropped
sectors agree; the batched form runs on such meshes; unsupported requests are
refused.
"""
import time

import numpy as np
import pytest

from gpu_common import data_scaled_error, run_library, torch_cuda
from oracle import CwenoOracle, Options
from synthetic import kuhn_tet_mesh, tri_mesh

pytestmark = pytest.mark.gpu

CASES = {
    "tri13_M1_nv4": (lambda: tri_mesh(13, 0.15, 1001), 1, 4),
    "tri13_M2_nv5": (lambda: tri_mesh(13, 0.15, 1002), 2, 5),
    "tri14_M3_nv9": (lambda: tri_mesh(14, 0.15, 1003), 3, 9),
    "tri12_M4_nv3": (lambda: tri_mesh(12, 0.15, 1004), 4, 3),
    "tri12_M3_bounded": (lambda: tri_mesh(12, 0.15, 1005, periodic=False), 3, 4),
    "kuhn5_M1_nv5": (lambda: kuhn_tet_mesh(5, 0.1, 1006), 1, 5),
    "kuhn5_M2_nv5": (lambda: kuhn_tet_mesh(5, 0.1, 1007), 2, 5),
    "kuhn6_M3_nv5": (lambda: kuhn_tet_mesh(6, 0.1, 1008), 3, 5),
    "kuhn5_M2_bounded": (lambda: kuhn_tet_mesh(5, 0.1, 1009, periodic=False), 2, 3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_device_operators_match_host_operators(case):
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    mk, M, nv = CASES[case]
    m = mk()
    print(f"[gpu devops] {case}: {m.n_cells} cells", flush=True)
    t0 = time.perf_counter()
    host = C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops="both")
    t1 = time.perf_counter()
    dev = C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops="both", device_operators=True)
    t2 = time.perf_counter()
    print(f"[gpu devops]   registration host {t1 - t0:.3f} s, device {t2 - t1:.3f} s", flush=True)
    assert dev.n_dropped == host.n_dropped
    assert dev.gather_len == host.gather_len
    rng = np.random.default_rng(1010)
    Q = rng.normal(size=(nv, m.n_cells)) + 3.0 * (rng.random((1, m.n_cells)) < 0.3)
    st = host.tables()["stencil"]
    a = run_library(torch, host, Q, torch.float64)
    b = run_library(torch, dev, Q, torch.float64)
    assert np.array_equal(b["coeffs"][:, 0, :].view(np.int64), Q.view(np.int64))
    err = data_scaled_error(b["coeffs"], a["coeffs"], Q, st)
    print(f"[gpu devops]   FP64 device vs host operators {err:.2e}", flush=True)
    assert err <= 1e-13
    assert np.abs(b["omega"] - a["omega"]).max() <= 1e-9
    o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
    idx = np.arange(0, m.n_cells, 7)
    ref = o.reconstruct(Q, cells=idx)
    assert data_scaled_error(b["coeffs"][:, :, idx], ref["coeffs"], Q, st[idx]) <= 1e-12
    a32 = run_library(torch, host, Q, torch.float32, want_diag=False)
    b32 = run_library(torch, dev, Q, torch.float32, want_diag=False)
    err32 = data_scaled_error(b32["coeffs"], ref_all := a["coeffs"], Q, st)
    print(f"[gpu devops]   FP32 device operators vs FP64 {err32:.2e}", flush=True)
    assert err32 <= 2e-6
    assert data_scaled_error(a32["coeffs"], ref_all, Q, st) <= 2e-6


def test_batch_on_device_operator_meshes_and_refusals():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    ms = [tri_mesh(12, 0.15, 1020), kuhn_tet_mesh(5, 0.1, 1021)]
    meshes = [C.Mesh(m.vertices, m.cells, 2, periodic=m.box, ops="f32", device_operators=True) for m in ms]
    qs = [torch.randn((4, lm.n_cells), dtype=torch.float32, device="cuda:0") for lm in meshes]
    outs = [torch.empty((4, lm.n_basis, lm.n_cells), dtype=torch.float32, device="cuda:0") for lm in meshes]
    batch = C.Batch(meshes, [4, 4], dtype="f32")
    batch.run(qs, outs)
    torch.cuda.synchronize()
    for lm, q, o in zip(meshes, qs, outs):
        assert torch.equal(o, lm.reconstruct(q))
    m = ms[0]
    for kw in (dict(host_only=True), dict(ops="none"), dict(weno=True)):
        with pytest.raises(C.CwenoError):
            C.Mesh(m.vertices, m.cells, 2, periodic=m.box, device_operators=True, **kw)
    k = kuhn_tet_mesh(7, 0.1, 1022)
    with pytest.raises(C.CwenoError):            # 104-cell central stencils: more than one row per lane
        C.Mesh(k.vertices, k.cells, 4, periodic=k.box, device_operators=True)
