"""GPU tests of the serving loop (cweno_server_*).

Results must equal cweno_reconstruct on the same mesh bit for bit (the same
host precompute and kernels), alone and batched with other requests in one
launch, with and without evictions; served results match the FP64 oracle on
sampled cells (FP64 to 1e-12, FP32 to the FP32 bar 2e-6 of the data scale)
with evictions forced; admission can be held and queued requests cancelled;
a ticket is released once its final state is reported; bad requests are
refused.
"""
import numpy as np
import pytest

from gpu_common import torch_cuda
from oracle import CwenoOracle, Options
from synthetic import kuhn_tet_mesh, tri_mesh, workload_fields

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


@pytest.mark.parametrize("dtype,batched", [("f32", False), ("f64", False), ("f32", True), ("f64", True)])
def test_server_matches_reconstruct_bitwise(dtype, batched):
    """batched: admission is held while every request is queued, so that they
    leave together in one launch of the batched kernel."""
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    tdt, raw, direct = _setup(torch, C, dtype)
    srv = C.Server(1 << 32, dtype=dtype, max_inflight=4, n_streams=3, max_batch=64 if batched else 1)
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
    if batched:
        srv.pause(True)
    tickets = [srv.submit(i, q, o) for i, q, o in zip(ids, qs, outs)]
    srv.pause(False)
    for t in tickets:
        srv.wait(t, 30.0)
    for o, r in zip(outs, refs):
        assert torch.equal(o, r)
    st = srv.stats()
    assert st["completed"] == len(tickets) and st["evictions"] == 0 and st["uploads"] == len(ids)
    assert st["p50_s"] > 0 and st["p99_s"] >= st["p50_s"]
    ls = srv.launch_stats()
    if batched:
        assert ls["launches"] == 1 and ls["largest_launch"] == len(tickets) and ls["shared_requests"] == len(tickets)
    else:
        assert ls["launches"] == len(tickets) and ls["largest_launch"] == 1 and ls["shared_requests"] == 0
    assert ls["tickets_held"] == 0          # every ticket was reported by wait and released
    with pytest.raises(C.CwenoError) as ei:
        srv.poll(tickets[0])
    assert ei.value.name == "CWENO_E_ARG"


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_served_results_match_the_oracle_with_evictions(dtype):
    """A 2-D and a 3-D mesh served in a mix with evictions forced (budget below
    the sum of the images), batched and alone; sampled cells of every served
    result against the FP64 oracle."""
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    tdt = {"f64": torch.float64, "f32": torch.float32}[dtype]
    tol = 1e-12 if dtype == "f64" else 2e-6
    specs = [(tri_mesh(16, 0.15, 421), 3, "mhd2d"), (kuhn_tet_mesh(6, 0.1, 422), 3, "euler3d_blast"),
             (tri_mesh(12, 0.15, 423), 4, "smooth_jump"), (kuhn_tet_mesh(5, 0.1, 424), 2, "euler3d_blast")]
    probe = C.Server(1 << 32, dtype=dtype)
    sizes = [probe.mesh_info(probe.register(m.vertices, m.cells, M, periodic=m.box))["image_bytes"]
             for m, M, _ in specs]
    del probe
    budget = max(int(sum(sizes) * 0.6), int(max(sizes) * 1.05))
    srv = C.Server(budget, dtype=dtype, max_inflight=2, n_streams=2)
    ids = [srv.register(m.vertices, m.cells, M, periodic=m.box) for m, M, _ in specs]
    Qs = [workload_fields(m, f, 430 + k) for k, (m, M, f) in enumerate(specs)]
    rng = np.random.default_rng(431)
    order = [int(k) for k in rng.integers(0, len(specs), 24)]
    qs = [torch.tensor(Q, dtype=tdt, device="cuda:0") for Q in Qs]
    outs = [[torch.full((Q.shape[0], srv.mesh_info(i)["n_basis"], m.n_cells), float("nan"), dtype=tdt,
                        device="cuda:0") for _ in range(order.count(k))]
            for k, (i, Q, (m, _, _)) in enumerate(zip(ids, Qs, specs))]
    torch.cuda.synchronize()
    used = [0] * len(specs)
    tickets = []
    srv.pause(True)                        # the first half leaves in shared launches
    for n, k in enumerate(order):
        if n == len(order) // 2:
            srv.pause(False)
        tickets.append(srv.submit(ids[k], qs[k], outs[k][used[k]]))
        used[k] += 1
    for t in tickets:
        srv.wait(t, 60.0)
    st, ls = srv.stats(), srv.launch_stats()
    print(f"[gpu server oracle {dtype}] budget {budget} B of {sum(sizes)} B: {st} {ls}", flush=True)
    assert st["evictions"] > 0 and ls["shared_requests"] > 0
    for k, (m, M, _) in enumerate(specs):
        cells = np.sort(rng.choice(m.n_cells, size=min(40, m.n_cells), replace=False))
        o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
        ref = o.reconstruct(Qs[k], cells=cells)["coeffs"]
        st0 = np.array([o.stencils(int(i))[0] for i in cells])
        scale = np.maximum(np.abs(Qs[k][:, st0]).max(axis=2), 1e-300)[:, None, :]
        for out in outs[k]:
            got = out.cpu().numpy().astype(np.float64)
            assert np.array_equal(got[:, 0], qs[k].cpu().numpy().astype(np.float64))
            assert np.isfinite(got).all()
            err = float((np.abs(got[:, :, cells] - ref) / scale).max())
            assert err <= tol, (k, err)


@pytest.mark.parametrize("pinned", [True, False])
def test_server_evicts_under_a_small_budget(pinned):
    """pinned=False: a pinned limit of 0, so every image is pageable."""
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    tdt, raw, direct = _setup(torch, C, "f32")
    # measure the images with a roomy server, then serve with room for about half of them
    probe = C.Server(1 << 32, dtype="f32")
    sizes = [probe.mesh_info(probe.register(m.vertices, m.cells, M, periodic=m.box))["image_bytes"] for m, M in raw]
    del probe
    budget = max(int(sum(sizes) * 0.5), int(max(sizes) * 1.05))
    srv = C.Server(budget, dtype="f32", max_inflight=3, n_streams=2)
    if not pinned:
        srv.set_pinned_limit(0)
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
        srv.cancel(t[0])                           # finished (and released): cannot cancel
    assert srv.launch_stats()["tickets_held"] == 0
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
