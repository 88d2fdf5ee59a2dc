"""The batch workload at full size: 64 uneven meshes in one graph launch.

The seeded recipe (synthetic.batch_spec): cell counts log-uniform on
[1e3, 3e5] (about 3.4 million cells in all), dimension 2 or 3, degree 2, 3
or 4, d + 2 variables of smooth fields with a planar or spherical jump.  The
FP32 batch (the form the benchmark times) and the FP64 batch both run; every
mesh is checked against the FP64 oracle at sampled cells (FP64 to 1e-12, FP32
to the single-precision bar of test_gpu_fp32_and_full), and at every cell for
a bitwise coefficient 0 and finite values.
"""
import numpy as np
import pytest

from gpu_common import torch_cuda
from oracle import CwenoOracle, Options
from synthetic import batch_spec, workload_fields, workload_mesh

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 2e-6


@pytest.mark.timeout(900)
def test_batch64_every_mesh_against_oracle():
    torch = torch_cuda()
    import paper_1612_09335_amd as C
    spec = batch_spec()
    print(f"[gpu batch64] building {len(spec)} meshes", flush=True)
    raw = [(workload_mesh(d, n, sd), M, sd) for d, n, M, sd in spec]
    Qs = [workload_fields(m, "smooth_jump", sd) for m, M, sd in raw]
    meshes = [C.Mesh(m.vertices, m.cells, M, periodic=m.box, ops="both") for m, M, sd in raw]
    print(f"[gpu batch64] {sum(m.n_cells for m, _, _ in raw)} cells registered", flush=True)
    # oracle values at sampled cells of every mesh
    refs = []
    for t, ((m, M, sd), Q) in enumerate(zip(raw, Qs)):
        rng = np.random.default_rng(sd)
        idx = np.unique(np.concatenate([rng.choice(m.n_cells, 12, replace=False), [m.n_cells - 1]]))
        o = CwenoOracle(m.vertices, m.cells, m.box, Options(degree=M))
        refs.append((idx, o.reconstruct(Q, cells=idx)["coeffs"]))
    print("[gpu batch64] oracle done", flush=True)
    for tag, tdt, tol in (("f32", torch.float32, TOL32), ("f64", torch.float64, TOL64)):
        qs = [torch.tensor(Q, dtype=tdt, device="cuda:0") for Q in Qs]
        outs = [torch.full((Q.shape[0], lm.n_basis, lm.n_cells), float("nan"), dtype=tdt, device="cuda:0")
                for lm, Q in zip(meshes, Qs)]
        batch = C.Batch(meshes, [Q.shape[0] for Q in Qs], dtype=tag)
        batch.run(qs, outs)
        batch.run(qs, outs)        # a replay computes the same
        torch.cuda.synchronize()
        worst = 0.0
        for (m, M, sd), lm, Q, o, (idx, want) in zip(raw, meshes, Qs, outs, refs):
            got = o.cpu().numpy().astype(np.float64)
            assert np.isfinite(got).all()
            assert np.array_equal(got[:, 0, :], Q.astype(np.float32 if tag == "f32" else np.float64))
            st = lm.tables()["stencil"][idx]
            scale = np.maximum(np.abs(Q[:, st]).max(axis=2), 1e-300)
            err = (np.abs(got[:, :, idx] - want) / scale[:, None, :]).max()
            worst = max(worst, err)
            assert err <= tol, (tag, m.name, M, err)
        print(f"[gpu batch64] {tag}: worst sampled data-scaled error {worst:.3e}", flush=True)
        del batch, qs, outs
