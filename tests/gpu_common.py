"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def data_scaled_error(got, want, Q, stencils):
    """max over (v, l, cell) of |got - want| / max_{j in S0(cell)} |Q[v, j]|.

    got/want: [nv, nb, n] coefficients of the same cells; stencils [n, n_e]."""
    scale = np.abs(Q[:, stencils]).max(axis=2)               # [nv, n]
    scale = np.maximum(scale, 1e-300)
    return (np.abs(got - want) / scale[:, None, :]).max()


def run_library(torch, mesh_lib, Q, dtype, want_diag=True):
    dev = torch.device("cuda:0")
    q = torch.tensor(Q, dtype=dtype, device=dev).contiguous()
    nv = Q.shape[0]
    d = mesh_lib.dim
    sig = torch.full((nv, d + 2, mesh_lib.n_cells), float("nan"), dtype=dtype, device=dev) if want_diag else None
    om = torch.full((nv, d + 2, mesh_lib.n_cells), float("nan"), dtype=dtype, device=dev) if want_diag else None
    out = torch.full((nv, mesh_lib.n_basis, mesh_lib.n_cells), float("nan"), dtype=dtype, device=dev)
    mesh_lib.reconstruct(q, out=out, sigma=sig, omega=om)
    torch.cuda.synchronize()
    res = dict(coeffs=out.cpu().numpy().astype(np.float64), q=q.cpu().numpy())
    if want_diag:
        res["sigma"] = sig.cpu().numpy().astype(np.float64)
        res["omega"] = om.cpu().numpy().astype(np.float64)
    return res
