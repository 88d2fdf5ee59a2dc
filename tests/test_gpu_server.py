"""GPU tests of the serving loop (cweno_server_*).

Results must equal cweno_reconstruct on the same mesh bit for bit (the same
host precompute and kernels), with and without evictions; admission can be
held and queued requests cancelled; bad requests are refused.
"""
import numpy as np
import pytest

from gpu_common import torch_cuda
from synthetic import kuhn_tet_mesh, tri_mesh

pytestmark = pytest.mark.gpu

MESHES = [(lambda: tri_mesh(12, 0.15, 401), 3), (lambda: tri_mesh(9, 0.15, 402), 2),
          (lambda: kuhn_tet_mesh(5, 0.1, 403), 2), (lambda: tri_mesh(14, 0.15, 404), 4),
          (lambda: kuhn_tet_mesh(6, 0.1, 405), 3)]


def _setup(torch, C, dtype):
    tdt = {"f64": torch.float64, "f32": torch.float32}[dtype]
    raw = [(mk(), M) for mk, M in MESHES]
    direct = [C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops=dtype) for m, M in raw]
    return tdt, raw, direct


def _register_all(srv, raw):
    return [srv.register(m.vertices, m.cells, M, periodic=m.box) for m, M in raw]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_server_matches_reconstruct_bitwise(dtype):
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    tdt, raw, direct = _setup(torch, C, dtype)
    srv = C.Server(1 << 32, dtype=dtype, max_inflight=4, n_streams=3)
    ids = _register_all(srv, raw)
    rng = np.random.default_rng(7)
    qs, outs, refs = [], [], []
    for (m, M), lm in zip(raw, direct):
        nv = int(rng.integers(1, 8))
        q = torch.tensor(rng.normal(size=(nv, m.n_cells)), dtype=tdt, device="cuda:0")
        qs.append(q)
        outs.append(torch.full((nv, lm.n_basis, lm.n_cells), float("nan"), dtype=tdt, device="cuda:0"))
        refs.append(lm.reconstruct(q))
    torch.cuda.synchronize()
    tickets = [srv.submit(i, q, o) for i, q, o in zip(ids, qs, outs)]
    for t in tickets:
        srv.wait(t, 30.0)
        assert srv.poll(t)
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["evictions"] == 0 and st["uploads"] == len(ids)
    assert st["p50_s"] > 0 and st["p99_s"] >= st["p50_s"]


def test_server_evicts_under_a_small_budget():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    tdt, raw, direct = _setup(torch, C, "f32")
    # measure the images with a roomy server, then serve with room for about half of them
    probe = C.Server(1 << 32, dtype="f32")
    sizes = [probe.mesh_info(probe.register(m.vertices, m.cells, M, periodic=m.box))["image_bytes"] for m, M in raw]
    del probe
    budget = max(int(sum(sizes) * 0.5), int(max(sizes) * 1.05))
    srv = C.Server(budget, dtype="f32", max_inflight=3, n_streams=2)
    ids = _register_all(srv, raw)
    rng = np.random.default_rng(8)
    order = [int(k) for k in rng.integers(0, len(ids), 60)]
    qs = [torch.tensor(rng.normal(size=(4, m.n_cells)), dtype=tdt, device="cuda:0") for m, _ in raw]
    refs = [lm.reconstruct(q) for lm, q in zip(direct, qs)]
    outs = [torch.full_like(r, float("nan")) for r in refs]
    torch.cuda.synchronize()
    for rnd in range(0, len(order), 10):
        chunk = order[rnd:rnd + 10]
        for k in set(chunk):
            outs[k].fill_(float("nan"))
        torch.cuda.synchronize()
        # requests of one mesh within a chunk write identical values to the same buffer
        tickets = [srv.submit(ids[k], qs[k], outs[k]) for k in chunk]
        for t in tickets:
            srv.wait(t, 30.0)
        for k in set(chunk):
            assert torch.equal(outs[k], refs[k]), k
    st = srv.stats()
    print(f"[gpu server] budget {budget} B: {st}", flush=True)
    assert st["completed"] == len(order)
    assert st["evictions"] > 0 and st["uploads"] > len(ids)


def test_server_pause_cancel_and_errors():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    m = tri_mesh(10, 0.15, 410)
    lm = C.Mesh(m.vertices, m.cells, 2, periodic=m.box, ops="f32")
    srv = C.Server(1 << 30, dtype="f32", max_inflight=2)
    mid = srv.register(m.vertices, m.cells, 2, periodic=m.box)
    q = torch.ones((3, m.n_cells), dtype=torch.float32, device="cuda:0")
    outs = [torch.zeros((3, lm.n_basis, lm.n_cells), dtype=torch.float32, device="cuda:0") for _ in range(3)]
    torch.cuda.synchronize()
    srv.pause(True)
    t = [srv.submit(mid, q, o) for o in outs]
    assert not srv.poll(t[1])
    srv.cancel(t[1])
    with pytest.raises(C.CwenoError) as ei:
        srv.poll(t[1])
    assert ei.value.name == "CWENO_E_CANCELLED"
    with pytest.raises(C.CwenoError) as ei:
        srv.wait(t[0], 0.05)                       # held: times out
    assert ei.value.name == "CWENO_E_BUSY"
    srv.pause(False)
    srv.wait(t[0], 30.0)
    srv.wait(t[2], 30.0)
    ref = lm.reconstruct(q)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], ref) and torch.equal(outs[2], ref)
    assert torch.count_nonzero(outs[1]) == 0       # the cancelled request never ran
    with pytest.raises(C.CwenoError):
        srv.cancel(t[0])                           # finished: cannot cancel
    # unknown mesh, wrong precision, image larger than the budget
    import ctypes
    tk = ctypes.c_int64()
    assert C.lib.cweno_server_submit(srv._h, mid + 5, 3, C.F32, q.data_ptr(), outs[0].data_ptr(),
                                     ctypes.byref(tk)) == -1
    assert C.lib.cweno_server_submit(srv._h, mid, 3, C.F64, q.data_ptr(), outs[0].data_ptr(),
                                     ctypes.byref(tk)) == -1
    small = C.Server(1 << 12, dtype="f32")
    with pytest.raises(C.CwenoError) as ei:
        small.register(m.vertices, m.cells, 2, periodic=m.box)
    assert ei.value.name == "CWENO_E_BUDGET"
