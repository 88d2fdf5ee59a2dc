"""MI355X CWENO reconstruction on unstructured simplex meshes (arXiv 1612.09335).

Thin Python binding of the C ABI in ``include/cweno.h``: argument marshalling
only.  Every step of the reconstruction runs in ``libcweno.so`` (host
precompute in C++, reconstruction in gfx950 HIP kernels); PyTorch tensors
provide device memory and streams.  There is no fallback: if the library is
missing, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcweno.so")

F64, F32 = 0, 1
OPS = {"f64": 0, "f32": 1, "both": 2, "none": 3}
SECTOR_RULES = {"cone": 0, "face": 1}
FLAG_HOST_ONLY, FLAG_SIGMA0_POPT, FLAG_LINEAR_WEIGHTS, FLAG_MOVING, FLAG_WENO, FLAG_DEVICE_OPERATORS = 1, 2, 4, 8, 16, 32

STATUS = {0: "CWENO_OK", -1: "CWENO_E_ARG", -2: "CWENO_E_MESH", -3: "CWENO_E_STENCIL",
          -4: "CWENO_E_RANK", -5: "CWENO_E_PERIODIC", -6: "CWENO_E_NOMEM", -7: "CWENO_E_BUDGET",
          -8: "CWENO_E_HIP", -9: "CWENO_E_BUSY", -10: "CWENO_E_CANCELLED"}

SYMBOLS = ("cweno_mesh_create", "cweno_mesh_destroy", "cweno_mesh_info", "cweno_mesh_tables",
           "cweno_mesh_operators", "cweno_mesh_weno_tables", "cweno_reconstruct", "cweno_reconstruct_moving",
           "cweno_mesh_set_moving_shape", "cweno_mesh_moving_shape", "cweno_points_create",
           "cweno_points_basis", "cweno_points_destroy", "cweno_evaluate", "cweno_reconstruct_points",
           "cweno_status_string",
           "cweno_last_error",
           "cweno_abi_version", "cweno_num_variants", "cweno_mesh_set_variant", "cweno_mesh_get_variant",
           "cweno_mesh_tune", "cweno_batch_create", "cweno_batch_run", "cweno_batch_info", "cweno_batch_group",
           "cweno_batch_destroy", "cweno_batch_run_noalloc", "cweno_server_create", "cweno_server_register", "cweno_server_register_mesh",
           "cweno_server_mesh_info", "cweno_server_submit", "cweno_server_poll", "cweno_server_wait", "cweno_server_cancel",
           "cweno_server_stats", "cweno_server_reset_stats", "cweno_server_set_batch", "cweno_server_set_pinned_limit",
           "cweno_server_launch_stats", "cweno_server_pause", "cweno_server_destroy")


class CwenoError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {detail}")


class _Options(ctypes.Structure):
    _fields_ = [("periodic", ctypes.c_double * 3), ("stencil_factor", ctypes.c_double),
                ("lambda0", ctypes.c_double), ("eps", ctypes.c_double), ("r", ctypes.c_int),
                ("ops", ctypes.c_int), ("sector_rule", ctypes.c_int), ("flags", ctypes.c_uint)]


def _load():
    # torch bundles its own HIP runtime with the same soname as ROCm's; loading
    # torch first makes the library bind to that runtime, so device pointers
    # and streams are shared by one runtime instance in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1612_09335_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32p = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)
    lib.cweno_mesh_create.argtypes = [ctypes.c_int, i64, vp, i64, vp, ctypes.c_int, ctypes.POINTER(_Options),
                                      vp, ctypes.POINTER(vp)]
    lib.cweno_mesh_destroy.argtypes = [vp]
    lib.cweno_mesh_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.cweno_mesh_tables.argtypes = [vp, vp, vp, vp]
    lib.cweno_mesh_operators.argtypes = [vp, i64, vp, vp, vp]
    lib.cweno_reconstruct.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp]
    lib.cweno_reconstruct_moving.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp]
    lib.cweno_mesh_set_moving_shape.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.cweno_mesh_moving_shape.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.cweno_mesh_weno_tables.argtypes = [vp, ctypes.POINTER(ctypes.c_int), vp]
    lib.cweno_points_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.cweno_points_basis.argtypes = [vp, vp]
    lib.cweno_points_destroy.argtypes = [vp]
    lib.cweno_evaluate.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.cweno_reconstruct_points.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
    lib.cweno_mesh_set_variant.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.cweno_mesh_get_variant.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.cweno_mesh_tune.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp,
                                    ctypes.POINTER(ctypes.c_double)]
    lib.cweno_status_string.argtypes = [ctypes.c_int]
    lib.cweno_status_string.restype = ctypes.c_char_p
    lib.cweno_last_error.restype = ctypes.c_char_p
    lib.cweno_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                       ctypes.c_char_p, vp, ctypes.POINTER(vp)]
    lib.cweno_batch_run.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.cweno_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(i64),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.cweno_batch_group.argtypes = [vp, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 7 + [
        ctypes.POINTER(ctypes.c_double)]
    lib.cweno_batch_destroy.argtypes = [vp]
    lib.cweno_batch_run_noalloc.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int),
                                            ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    i64p = ctypes.POINTER(i64)
    lib.cweno_server_create.argtypes = [i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    lib.cweno_server_register.argtypes = [vp, ctypes.c_int, i64, vp, i64, vp, ctypes.c_int, ctypes.POINTER(_Options),
                                          i64p]
    lib.cweno_server_register_mesh.argtypes = [vp, vp, i64p]
    lib.cweno_server_mesh_info.argtypes = [vp, i64, i64p, ctypes.POINTER(ctypes.c_int), i64p,
                                           ctypes.POINTER(ctypes.c_int)]
    lib.cweno_server_submit.argtypes = [vp, i64, ctypes.c_int, ctypes.c_int, vp, vp, i64p]
    lib.cweno_server_poll.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_int)]
    lib.cweno_server_wait.argtypes = [vp, i64, ctypes.c_double]
    lib.cweno_server_cancel.argtypes = [vp, i64]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.cweno_server_stats.argtypes = [vp, dp, dp, dp, i64p, i64p, i64p, i64p]
    lib.cweno_server_reset_stats.argtypes = [vp]
    lib.cweno_server_set_batch.argtypes = [vp, ctypes.c_int]
    lib.cweno_server_set_pinned_limit.argtypes = [vp, i64]
    lib.cweno_server_launch_stats.argtypes = [vp, i64p, i64p, i64p, i64p]
    lib.cweno_server_pause.argtypes = [vp, ctypes.c_int]
    lib.cweno_server_destroy.argtypes = [vp]
    for name in ("cweno_mesh_create", "cweno_mesh_destroy", "cweno_mesh_info", "cweno_mesh_tables",
                 "cweno_mesh_operators", "cweno_mesh_weno_tables", "cweno_reconstruct", "cweno_mesh_set_variant",
                 "cweno_mesh_get_variant", "cweno_mesh_tune", "cweno_num_variants", "cweno_batch_create",
                 "cweno_batch_run", "cweno_batch_info", "cweno_batch_group", "cweno_batch_destroy",
                 "cweno_batch_run_noalloc",
                 "cweno_server_create", "cweno_server_register", "cweno_server_register_mesh",
                 "cweno_server_mesh_info", "cweno_server_submit",
                 "cweno_server_poll", "cweno_server_wait", "cweno_server_cancel", "cweno_server_stats",
                 "cweno_server_reset_stats", "cweno_server_set_batch", "cweno_server_set_pinned_limit",
                 "cweno_server_launch_stats",
                 "cweno_server_pause", "cweno_server_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def _check(st: int):
    if st != 0:
        raise CwenoError(st, lib.cweno_last_error().decode())


def n_basis(M: int, d: int) -> int:
    """eq. cwenoM: (1/d!) prod_{l=1..d} (M + l)."""
    return (M + 1) * (M + 2) // 2 if d == 2 else (M + 1) * (M + 2) * (M + 3) // 6


class Mesh:
    """A registered mesh with its reconstruction operators (cweno_mesh_create)."""

    def __init__(self, vertices, cells, degree: int, periodic=(0.0, 0.0, 0.0), stencil_factor: float = 0.0,
                 lambda0: float = 0.0, eps: float = 0.0, r: int = 0, ops: str = "f64",
                 sector_rule: str = "cone", sigma0_popt: bool = False, linear_weights: bool = False,
                 host_only: bool = False, moving: bool = False, weno: bool = False,
                 device_operators: bool = False, stream=None):
        V = np.ascontiguousarray(vertices, dtype=np.float64)
        C = np.ascontiguousarray(cells, dtype=np.int32)
        self.dim = int(V.shape[1])
        self.degree = int(degree)
        o = _Options()
        for a, L in enumerate(tuple(periodic)[:3]):
            o.periodic[a] = float(L)
        o.stencil_factor = float(stencil_factor)
        o.lambda0 = float(lambda0)
        o.eps = float(eps)
        o.r = int(r)
        o.ops = OPS[ops]
        o.sector_rule = SECTOR_RULES[sector_rule]
        o.flags = ((FLAG_HOST_ONLY if host_only else 0) | (FLAG_SIGMA0_POPT if sigma0_popt else 0)
                   | (FLAG_LINEAR_WEIGHTS if linear_weights else 0) | (FLAG_MOVING if moving else 0)
                   | (FLAG_WENO if weno else 0) | (FLAG_DEVICE_OPERATORS if device_operators else 0))
        self.weno = weno
        self.n_vertices = int(V.shape[0])
        self.moving = moving
        self.ops = ops
        self.host_only = host_only
        h = ctypes.c_void_p()
        st = lib.cweno_mesh_create(self.dim, V.shape[0], V.ctypes.data, C.shape[0], C.ctypes.data,
                                   self.degree, ctypes.byref(o), _stream_ptr(stream), ctypes.byref(h))
        _check(st)
        self._h = h
        n, nb, ne, g, db, nd = (ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(),
                                ctypes.c_int64(), ctypes.c_int64())
        _check(lib.cweno_mesh_info(h, ctypes.byref(n), ctypes.byref(nb), ctypes.byref(ne), ctypes.byref(g),
                                   ctypes.byref(db), ctypes.byref(nd)))
        self.n_cells, self.n_basis, self.n_e = n.value, nb.value, ne.value
        self.gather_len, self.device_bytes, self.n_dropped = g.value, db.value, nd.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.cweno_mesh_destroy(h)
            self._h = None

    def tables(self):
        """Host copies: face_nbr [n, d+1], stencil [n, n_e], sectors [n, d+1, d+1]."""
        d = self.dim
        fn = np.empty((self.n_cells, d + 1), dtype=np.int32)
        st = np.empty((self.n_cells, self.n_e), dtype=np.int32)
        se = np.empty((self.n_cells, d + 1, d + 1), dtype=np.int32)
        _check(lib.cweno_mesh_tables(self._h, fn.ctypes.data, st.ctypes.data, se.ctypes.data))
        return dict(face_nbr=fn, stencil=st, sectors=se)

    def weno_tables(self):
        """Classical-WENO stencils [n_cells, n_s, n_e] (rows of -1: unfillable)."""
        ns = ctypes.c_int()
        _check(lib.cweno_mesh_weno_tables(self._h, ctypes.byref(ns), None))
        st = np.empty((self.n_cells, ns.value, self.n_e), dtype=np.int32)
        _check(lib.cweno_mesh_weno_tables(self._h, None, st.ctypes.data))
        return st

    def operators(self, cell: int):
        """FP64 operators of one cell: pinv [nb-1, n_e-1], binv [d+1, d, d], sigma [nb-1, nb-1]."""
        d, nb, ne = self.dim, self.n_basis, self.n_e
        P = np.empty((nb - 1, ne - 1))
        B = np.empty((d + 1, d, d))
        S = np.empty((nb - 1, nb - 1))
        _check(lib.cweno_mesh_operators(self._h, int(cell), P.ctypes.data, B.ctypes.data, S.ctypes.data))
        return P, B, S

    def sigma_matrix(self):
        nb = self.n_basis
        S = np.empty((nb - 1, nb - 1))
        _check(lib.cweno_mesh_operators(self._h, 0, None, None, S.ctypes.data))
        return S

    def reconstruct(self, q, out=None, sigma=None, omega=None, stream=None):
        """cweno_reconstruct on torch CUDA tensors: q [n_vars, n_cells] -> coeffs [n_vars, n_basis, n_cells].

        ``sigma`` / ``omega`` may be preallocated [n_vars, d+2, n_cells] tensors (or None).
        Asynchronous on ``stream`` (a torch stream; None = torch's current stream).
        """
        import torch
        if not q.is_cuda or q.dim() != 2 or q.shape[1] != self.n_cells or not q.is_contiguous():
            raise ValueError("q must be a contiguous CUDA tensor [n_vars, n_cells]")
        dt = {torch.float64: F64, torch.float32: F32}.get(q.dtype)
        if dt is None:
            raise ValueError("q must be float64 or float32")
        nv = q.shape[0]
        if out is None:
            out = torch.empty((nv, self.n_basis, self.n_cells), dtype=q.dtype, device=q.device)
        for t, shape in ((out, (nv, self.n_basis, self.n_cells)), (sigma, (nv, self.dim + 2, self.n_cells)),
                         (omega, (nv, self.dim + 2, self.n_cells))):
            if t is not None and (tuple(t.shape) != shape or t.dtype != q.dtype or not t.is_contiguous()
                                  or t.device != q.device):
                raise ValueError(f"output tensor must be contiguous {q.dtype} {shape} on {q.device}")
        if stream is None:
            stream = torch.cuda.current_stream(q.device)
        _check(lib.cweno_reconstruct(self._h, nv, dt, q.data_ptr(), out.data_ptr(),
                                     None if sigma is None else sigma.data_ptr(),
                                     None if omega is None else omega.data_ptr(), _stream_ptr(stream)))
        return out

    def reconstruct_moving(self, vertices, q, out=None, sigma=None, omega=None, fault=None, stream=None):
        """cweno_reconstruct_moving: operators rebuilt from ``vertices`` (CUDA float64
        [n_vertices, dim]) for this call; otherwise as ``reconstruct``.  ``fault`` may be
        a CUDA int32 tensor of one element that the kernel ORs its fault bits into."""
        import torch
        if not q.is_cuda or q.dim() != 2 or q.shape[1] != self.n_cells or not q.is_contiguous():
            raise ValueError("q must be a contiguous CUDA tensor [n_vars, n_cells]")
        if (not vertices.is_cuda or vertices.dtype != torch.float64 or not vertices.is_contiguous()
                or tuple(vertices.shape) != (self.n_vertices, self.dim)):
            raise ValueError(f"vertices must be a contiguous CUDA float64 tensor [{self.n_vertices}, {self.dim}]")
        dt = {torch.float64: F64, torch.float32: F32}.get(q.dtype)
        if dt is None:
            raise ValueError("q must be float64 or float32")
        nv = q.shape[0]
        if out is None:
            out = torch.empty((nv, self.n_basis, self.n_cells), dtype=q.dtype, device=q.device)
        for t, shape in ((out, (nv, self.n_basis, self.n_cells)), (sigma, (nv, self.dim + 2, self.n_cells)),
                         (omega, (nv, self.dim + 2, self.n_cells))):
            if t is not None and (tuple(t.shape) != shape or t.dtype != q.dtype or not t.is_contiguous()
                                  or t.device != q.device):
                raise ValueError(f"output tensor must be contiguous {q.dtype} {shape} on {q.device}")
        if fault is not None and (not fault.is_cuda or fault.dtype != torch.int32 or fault.numel() < 1):
            raise ValueError("fault must be a CUDA int32 tensor")
        if stream is None:
            stream = torch.cuda.current_stream(q.device)
        _check(lib.cweno_reconstruct_moving(self._h, vertices.data_ptr(), nv, dt, q.data_ptr(), out.data_ptr(),
                                            None if sigma is None else sigma.data_ptr(),
                                            None if omega is None else omega.data_ptr(),
                                            None if fault is None else fault.data_ptr(), _stream_ptr(stream)))
        return out

    def set_moving_shape(self, seg, rpl):
        """cweno_mesh_set_moving_shape: the moving kernel's work mapping (seg lanes per
        cell, rpl stencil rows per lane); (0, 0) restores the default."""
        _check(lib.cweno_mesh_set_moving_shape(self._h, int(seg), int(rpl)))

    def moving_shape(self):
        """cweno_mesh_moving_shape: (seg, rpl) of the next moving-mesh call."""
        seg, rpl = ctypes.c_int(), ctypes.c_int()
        _check(lib.cweno_mesh_moving_shape(self._h, ctypes.byref(seg), ctypes.byref(rpl)))
        return seg.value, rpl.value

    def evaluate(self, points, coeffs, out=None, stream=None):
        """cweno_evaluate: coeffs [n_vars, n_basis, n_cells] -> values [n_vars, n_points, n_cells]."""
        import torch
        if (not coeffs.is_cuda or coeffs.dim() != 3 or tuple(coeffs.shape[1:]) != (self.n_basis, self.n_cells)
                or not coeffs.is_contiguous()):
            raise ValueError("coeffs must be a contiguous CUDA tensor [n_vars, n_basis, n_cells]")
        dt = {torch.float64: F64, torch.float32: F32}.get(coeffs.dtype)
        if dt is None:
            raise ValueError("coeffs must be float64 or float32")
        nv = coeffs.shape[0]
        shape = (nv, points.n_points, self.n_cells)
        if out is None:
            out = torch.empty(shape, dtype=coeffs.dtype, device=coeffs.device)
        elif tuple(out.shape) != shape or out.dtype != coeffs.dtype or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous {coeffs.dtype} tensor {shape}")
        if stream is None:
            stream = torch.cuda.current_stream(coeffs.device)
        _check(lib.cweno_evaluate(self._h, points._h, nv, dt, coeffs.data_ptr(), out.data_ptr(),
                                  _stream_ptr(stream)))
        return out

    def reconstruct_points(self, points, q, out=None, stream=None):
        """cweno_reconstruct_points: q [n_vars, n_cells] -> values [n_vars, n_points, n_cells]."""
        import torch
        if not q.is_cuda or q.dim() != 2 or q.shape[1] != self.n_cells or not q.is_contiguous():
            raise ValueError("q must be a contiguous CUDA tensor [n_vars, n_cells]")
        dt = {torch.float64: F64, torch.float32: F32}.get(q.dtype)
        if dt is None:
            raise ValueError("q must be float64 or float32")
        shape = (q.shape[0], points.n_points, self.n_cells)
        if out is None:
            out = torch.empty(shape, dtype=q.dtype, device=q.device)
        elif tuple(out.shape) != shape or out.dtype != q.dtype or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous {q.dtype} tensor {shape}")
        if stream is None:
            stream = torch.cuda.current_stream(q.device)
        _check(lib.cweno_reconstruct_points(self._h, points._h, q.shape[0], dt, q.data_ptr(), out.data_ptr(),
                                            _stream_ptr(stream)))
        return out

    # ---------------------------------------------------------------- variants
    def set_variant(self, dtype: str, vb: int, variant: int):
        _check(lib.cweno_mesh_set_variant(self._h, {"f64": F64, "f32": F32}[dtype], vb, variant))

    def get_variant(self, dtype: str, vb: int):
        """(variant index, kind: 0 direct gathers / 1 LDS halo, stencil chunk KC)."""
        k, kind, kc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.cweno_mesh_get_variant(self._h, {"f64": F64, "f32": F32}[dtype], vb, ctypes.byref(k),
                                          ctypes.byref(kind), ctypes.byref(kc)))
        return k.value, kind.value, kc.value

    def tune(self, q, out=None, repeats: int = 5, stream=None) -> float:
        """cweno_mesh_tune on the given averages; returns the tuned time (ms)."""
        import torch
        dt = {torch.float64: F64, torch.float32: F32}[q.dtype]
        if out is None:
            out = torch.empty((q.shape[0], self.n_basis, self.n_cells), dtype=q.dtype, device=q.device)
        if stream is None:
            stream = torch.cuda.current_stream(q.device)
        ms = ctypes.c_double()
        _check(lib.cweno_mesh_tune(self._h, q.shape[0], dt, q.data_ptr(), out.data_ptr(), repeats,
                                   _stream_ptr(stream), ctypes.byref(ms)))
        return ms.value


class Points:
    """A registered set of reference points (cweno_points_create)."""

    def __init__(self, dim: int, degree: int, ref_points):
        P = np.ascontiguousarray(ref_points, dtype=np.float64)
        if P.ndim != 2 or P.shape[1] != dim:
            raise ValueError(f"ref_points must be [n_points, {dim}]")
        self.dim, self.degree, self.n_points = int(dim), int(degree), int(P.shape[0])
        self.ref_points = P
        h = ctypes.c_void_p()
        _check(lib.cweno_points_create(self.dim, self.degree, self.n_points, P.ctypes.data, ctypes.byref(h)))
        self._h = h

    def basis(self):
        """phi [n_points, n_basis]: the basis functions at the points (FP64, host)."""
        phi = np.empty((self.n_points, n_basis(self.degree, self.dim)))
        _check(lib.cweno_points_basis(self._h, phi.ctypes.data))
        return phi

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.cweno_points_destroy(h)
            self._h = None


def num_variants() -> int:
    return lib.cweno_num_variants()


class Batch:
    """Many meshes reconstructed by one graph launch (cweno_batch_create / cweno_batch_run).

    ``meshes``: device ``Mesh`` objects holding operators of ``dtype``; ``n_vars[i]``
    variables per run for mesh i.  The meshes are kept alive by the batch.
    """

    def __init__(self, meshes, n_vars, dtype: str = "f32", tune_cache: str | None = None, stream=None):
        self.meshes = list(meshes)
        self.n_vars = [int(v) for v in n_vars]
        if len(self.n_vars) != len(self.meshes):
            raise ValueError("one n_vars entry per mesh")
        self.dtype = dtype
        n = len(self.meshes)
        arr = (ctypes.c_void_p * n)(*[m._h.value for m in self.meshes])
        nv = (ctypes.c_int * n)(*self.n_vars)
        h = ctypes.c_void_p()
        _check(lib.cweno_batch_create(n, arr, nv, {"f64": F64, "f32": F32}[dtype],
                                      None if tune_cache is None else tune_cache.encode(), _stream_ptr(stream),
                                      ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.cweno_batch_destroy(h)
            self._h = None

    def run(self, qs, outs, stream=None):
        """q_i [n_vars_i, n_cells_i] -> outs_i [n_vars_i, n_basis_i, n_cells_i] (torch CUDA tensors)."""
        import torch
        tdt = {"f64": torch.float64, "f32": torch.float32}[self.dtype]
        n = len(self.meshes)
        if len(qs) != n or len(outs) != n:
            raise ValueError("one q and one out tensor per mesh")
        for m, v, q, o in zip(self.meshes, self.n_vars, qs, outs):
            if (q.dtype != tdt or not q.is_cuda or not q.is_contiguous() or tuple(q.shape) != (v, m.n_cells)
                    or o.dtype != tdt or not o.is_contiguous() or tuple(o.shape) != (v, m.n_basis, m.n_cells)):
                raise ValueError("q/out tensors must match each mesh's shape and the batch precision")
        if stream is None:
            stream = torch.cuda.current_stream(qs[0].device)
        qa = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
        oa = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        _check(lib.cweno_batch_run(self._h, qa, oa, _stream_ptr(stream)))
        return outs

    def info(self):
        ng, ni, ms = ctypes.c_int(), ctypes.c_int64(), ctypes.c_double()
        _check(lib.cweno_batch_info(self._h, ctypes.byref(ng), ctypes.byref(ni), ctypes.byref(ms)))
        groups = []
        for g in range(ng.value):
            vals = [ctypes.c_int() for _ in range(7)]
            gms = ctypes.c_double()
            _check(lib.cweno_batch_group(self._h, g, *[ctypes.byref(v) for v in vals], ctypes.byref(gms)))
            groups.append(dict(zip(("dim", "degree", "vb", "entries", "items", "variant", "grid"),
                                   [v.value for v in vals]), ms=gms.value))
        return dict(n_groups=ng.value, n_items=ni.value, tuned_ms=ms.value, groups=groups)


class Server:
    """Serving loop (cweno_server_*): registered meshes, HBM residency under a
    budget with least-recently-used eviction, requests batched as they arrive
    (max_inflight launches in flight, each carrying up to max_batch requests)."""

    def __init__(self, hbm_budget_bytes: int, dtype: str = "f32", max_inflight: int = 8, n_streams: int = 4,
                 max_batch: int = 64):
        self.dtype = dtype
        h = ctypes.c_void_p()
        _check(lib.cweno_server_create(int(hbm_budget_bytes), {"f64": F64, "f32": F32}[dtype], int(max_inflight),
                                       int(n_streams), ctypes.byref(h)))
        self._h = h
        self._meshes = {}
        self.set_batch(max_batch)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.cweno_server_destroy(h)
            self._h = None

    def register(self, vertices, cells, degree: int, periodic=(0.0, 0.0, 0.0), stencil_factor: float = 0.0,
                 lambda0: float = 0.0, eps: float = 0.0, r: int = 0, sector_rule: str = "cone") -> int:
        V = np.ascontiguousarray(vertices, dtype=np.float64)
        C = np.ascontiguousarray(cells, dtype=np.int32)
        o = _Options()
        for a, L in enumerate(tuple(periodic)[:3]):
            o.periodic[a] = float(L)
        o.stencil_factor, o.lambda0, o.eps, o.r = float(stencil_factor), float(lambda0), float(eps), int(r)
        o.sector_rule = SECTOR_RULES[sector_rule]
        mid = ctypes.c_int64()
        _check(lib.cweno_server_register(self._h, V.shape[1], V.shape[0], V.ctypes.data, C.shape[0], C.ctypes.data,
                                         int(degree), ctypes.byref(o), ctypes.byref(mid)))
        self._meshes[mid.value] = self.mesh_info(mid.value)
        return mid.value

    def register_mesh(self, mesh) -> int:
        """Register a ``Mesh`` built with host_only=True, reusing its precompute."""
        mid = ctypes.c_int64()
        _check(lib.cweno_server_register_mesh(self._h, mesh._h, ctypes.byref(mid)))
        self._meshes[mid.value] = self.mesh_info(mid.value)
        return mid.value

    def mesh_info(self, mesh_id: int):
        n, nb, ib, res = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int64(), ctypes.c_int()
        _check(lib.cweno_server_mesh_info(self._h, int(mesh_id), ctypes.byref(n), ctypes.byref(nb), ctypes.byref(ib),
                                          ctypes.byref(res)))
        return dict(n_cells=n.value, n_basis=nb.value, image_bytes=ib.value, resident=bool(res.value))

    def submit(self, mesh_id: int, q, out) -> int:
        """Queue a reconstruction of q [n_vars, n_cells] into out [n_vars, n_basis, n_cells] (torch CUDA)."""
        info = self._meshes[mesh_id]
        nv = q.shape[0]
        if (not q.is_cuda or not q.is_contiguous() or not out.is_contiguous() or q.dim() != 2
                or q.shape[1] != info["n_cells"] or tuple(out.shape) != (nv, info["n_basis"], info["n_cells"])
                or out.dtype != q.dtype):
            raise ValueError("q/out must be contiguous CUDA tensors matching the mesh")
        t = ctypes.c_int64()
        dt = F32 if str(q.dtype) == "torch.float32" else F64
        _check(lib.cweno_server_submit(self._h, int(mesh_id), nv, dt, q.data_ptr(), out.data_ptr(), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int()
        _check(lib.cweno_server_poll(self._h, int(ticket), ctypes.byref(done)))
        return bool(done.value)

    def wait(self, ticket: int, timeout_s: float = -1.0):
        _check(lib.cweno_server_wait(self._h, int(ticket), float(timeout_s)))

    def cancel(self, ticket: int):
        _check(lib.cweno_server_cancel(self._h, int(ticket)))

    def pause(self, paused: bool = True):
        _check(lib.cweno_server_pause(self._h, 1 if paused else 0))

    def stats(self):
        p50, p99, p999 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        c, e, u, ub = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.cweno_server_stats(self._h, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(p999),
                                      ctypes.byref(c), ctypes.byref(e), ctypes.byref(u), ctypes.byref(ub)))
        return dict(p50_s=p50.value, p99_s=p99.value, p999_s=p999.value, completed=c.value, evictions=e.value,
                    uploads=u.value, upload_bytes=ub.value)

    def reset_stats(self):
        _check(lib.cweno_server_reset_stats(self._h))

    def set_pinned_limit(self, nbytes: int):
        """Bytes of mesh images registered from now on that may be pinned (the rest pageable)."""
        _check(lib.cweno_server_set_pinned_limit(self._h, int(nbytes)))

    def set_batch(self, max_batch: int):
        """Requests one launch may carry (1: every request launched on its own)."""
        _check(lib.cweno_server_set_batch(self._h, int(max_batch)))

    def launch_stats(self):
        la, sh, big, held = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.cweno_server_launch_stats(self._h, ctypes.byref(la), ctypes.byref(sh), ctypes.byref(big),
                                             ctypes.byref(held)))
        return dict(launches=la.value, shared_requests=sh.value, largest_launch=big.value, tickets_held=held.value)


def batch_run_noalloc(meshes, qs, outs, dtype: str = "f64", stream=None):
    """cweno_batch_run_noalloc: the meshes' reconstructions as batched launches
    whose tables live in a static device array (no allocation).
    q_i [n_vars_i, n_cells_i] -> outs_i [n_vars_i, n_basis_i, n_cells_i] (torch CUDA tensors)."""
    import torch
    tdt = {"f64": torch.float64, "f32": torch.float32}[dtype]
    n = len(meshes)
    if len(qs) != n or len(outs) != n:
        raise ValueError("one q and one out tensor per mesh")
    for m, q, o in zip(meshes, qs, outs):
        if (q.dtype != tdt or not q.is_cuda or not q.is_contiguous() or q.dim() != 2 or q.shape[1] != m.n_cells
                or o.dtype != tdt or not o.is_contiguous() or tuple(o.shape) != (q.shape[0], m.n_basis, m.n_cells)):
            raise ValueError("q/out tensors must match each mesh's shape and the precision")
    if stream is None:
        stream = torch.cuda.current_stream(qs[0].device)
    ma = (ctypes.c_void_p * n)(*[m._h.value for m in meshes])
    nv = (ctypes.c_int * n)(*[q.shape[0] for q in qs])
    qa = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
    oa = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    _check(lib.cweno_batch_run_noalloc(n, ma, nv, {"f64": F64, "f32": F32}[dtype], qa, oa, _stream_ptr(stream)))
    return outs


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return getattr(stream, "cuda_stream", None)


__all__ = ["Mesh", "Points", "CwenoError", "n_basis", "batch_run_noalloc", "lib", "LIB_PATH", "SYMBOLS"]
