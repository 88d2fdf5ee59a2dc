"""Seeded synthetic workloads: simplex meshes and cell-average fields.

This package produces *inputs only*: vertex coordinates, cell connectivity and
cell averages of analytic test fields.  It holds none of the reconstruction's
arithmetic (no stencils, no basis, no least squares, no weights), so both the
CPU oracle and the GPU path may consume what it produces without sharing code.

The meshes mimic the paper's workloads (jittered periodic triangulations of the
unit square and Kuhn tetrahedrisations of the unit cube, Sec. 3); the fields
mimic its states (Euler variables with a Sod-type jump, Sec. 3.2; ideal-MHD
shaped nine-variable states, Sec. 3.3; a spherical blast).
"""
from .meshes import SimplexMesh, batch_spec, moved_vertices, tri_mesh, kuhn_tet_mesh, workload_mesh
from .fields import (cell_averages, euler2d_sod_circle, mhd2d_fourier_jump,
                     euler3d_blast, random_polynomial, polynomial_field,
                     smooth_fourier_field, workload_fields)

__all__ = [
    "SimplexMesh", "batch_spec", "moved_vertices", "tri_mesh", "kuhn_tet_mesh", "workload_mesh",
    "cell_averages", "euler2d_sod_circle", "mhd2d_fourier_jump",
    "euler3d_blast", "random_polynomial", "polynomial_field",
    "smooth_fourier_field", "workload_fields",
]
