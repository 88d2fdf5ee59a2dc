"""The oracle over many cells in a pool of single-threaded worker processes
(test helper, not collected by pytest).

Workers are spawned (a fresh interpreter: nothing of a parent's GPU state is
inherited and none of them touches the GPU), each builds its own oracle of the
mesh once, and the cells are split into one contiguous block per worker.  The
pool and multiprocessing's resource-tracker process are shut down before the
call returns.
"""
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

_STATE = None


def _init(vertices, cells, box, opts, Q):
    global _STATE
    from oracle import CwenoOracle
    _STATE = (CwenoOracle(vertices, cells, box, opts), Q)


def _reconstruct(ids):
    from threadpoolctl import threadpool_limits
    o, Q = _STATE
    with threadpool_limits(limits=1):
        r = o.reconstruct(Q, cells=ids)
    return r["coeffs"], r["omega"]


def _tables(ids):
    o, _ = _STATE
    t = o.tables(cells=ids)
    return t["stencil"], t["sectors"]


def workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _pool_map(fn, mesh, opts, Q, cells, n_workers):
    blocks = [b for b in np.array_split(np.asarray(cells, dtype=np.int64), n_workers or workers()) if len(b)]
    try:
        with ProcessPoolExecutor(len(blocks), mp_context=mp.get_context("spawn"), initializer=_init,
                                 initargs=(mesh.vertices, mesh.cells, mesh.box, opts, Q)) as pool:
            return list(pool.map(fn, [list(map(int, b)) for b in blocks]))
    finally:
        try:
            from multiprocessing import resource_tracker
            resource_tracker._resource_tracker._stop()
        except Exception:
            pass


def reconstruct(mesh, opts, Q, cells, n_workers=None):
    """Oracle coefficients [nv, nb, len(cells)] and weights [nv, d+2, len(cells)]."""
    parts = _pool_map(_reconstruct, mesh, opts, Q, cells, n_workers)
    return np.concatenate([p[0] for p in parts], axis=2), np.concatenate([p[1] for p in parts], axis=2)


def tables(mesh, opts, cells, n_workers=None):
    """Oracle central stencils [len(cells), n_e] and sectors [len(cells), d+1, d+1]."""
    parts = _pool_map(_tables, mesh, opts, None, cells, n_workers)
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])
