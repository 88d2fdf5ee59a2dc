"""CPU oracle for the CWENO reconstruction of Sec. 2.1 -- TEST INFRASTRUCTURE.

A plain, slow, FP64 implementation of what the library computes, written
from the paper and sharing no code with the library (no kernels, headers,
helpers, tables or generators).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the
library never falls back to it.

Parity status of each part (what pins it, from outside the oracle itself):

* basis        -- exact rational orthogonality, closed-form linear functions,
                  known Gram diagonals, degree count against the paper's DOF
                  totals (eq. cwenoM).
* Sigma        -- quadratic form equals sum_alpha int (d^alpha P)^2 from an
                  independent symbolic differentiation; closed form for
                  linear polynomials.
* quadrature   -- exact on monomials up to its degree.
* stencils     -- stencil sizes printed in the paper's stencil figures
                  (n_e = 12 in 2-D, 30 in 3-D at M = 2); brute-force
                  re-derivation of the ring rule; cone membership on hand-built
                  triangles.
* P_opt        -- polynomial reproduction on arbitrary meshes; brute-force
                  exact-rational KKT solve on tiny meshes.
* P_s, P0, w   -- linear data reproduced with omega = lambda; constant data
                  gives sigma = 0; exact-rational pipeline on tiny meshes;
                  conservation; convergence on smooth data; no overshoot at
                  jumps.
* dropped-sector rule -- the emptiness decision re-derived from exact
                  barycentric coordinates and brute-force hop distances; the
                  1e10 condition threshold decided exactly from the
                  characteristic polynomial of B^T B (collinear and
                  near-collinear hand-built sectors); the exact-rational
                  pipeline renormalising lambda on its own.
* options      -- face sector rule on a hand-built mesh and through the exact
                  pipeline; sigma_0 of P_opt through the exact pipeline.
* classical WENO (weno.py, the paper's comparison scheme) -- every stencil's
                  polynomial reproduces degree-M data, so the blend does;
                  conservation; cone and reverse-cone membership re-derived by
                  independent barycentric solves; stencil sizes; the weights
                  (default and the paper's pair, with dropped stencils)
                  against exact per-stencil KKT solves.
"""
from .basis import n_basis, sigma_matrix, evaluate as evaluate_basis, index_list
from .cweno import CwenoOracle, Options, linear_weights, stencil_size, evaluate_polynomial
from .stencils import StencilError, face_neighbours
from .weno import WenoOracle

__all__ = ["n_basis", "sigma_matrix", "evaluate_basis", "index_list", "CwenoOracle",
           "Options", "linear_weights", "stencil_size", "evaluate_polynomial",
           "StencilError", "face_neighbours", "WenoOracle"]
