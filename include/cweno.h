/*
 * cweno.h -- C ABI of the MI355X CWENO reconstruction library.
 *
 * The library implements the central WENO reconstruction of Dumbser,
 * Boscheri, Semplice and Russo, "Central WENO schemes for hyperbolic
 * conservation laws on fixed and moving unstructured meshes" (arXiv
 * 1612.09335), Sec. 2.1, on conforming triangle (d = 2) and tetrahedron
 * (d = 3) meshes with fixed (Eulerian) geometry: from the cell averages of
 * every variable it returns, per cell, the coefficients of one polynomial of
 * degree M that is defined everywhere in the cell (abstract; Sec. 2.1).
 *
 * Conventions
 *  - Every function returns a cweno_status: 0 on success, a negative code on
 *    failure.  Nothing throws across the ABI.  cweno_last_error() returns a
 *    human-readable detail of the calling thread's last failure.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device memory on the current device.  Streams are hipStream_t passed as
 *    void* (NULL = the default stream).
 *  - Cell c's reference frame is fixed by its vertex order: vertex 0 maps to
 *    the origin of the unit simplex and vertex k to the k-th unit vector
 *    (Sec. 2, eq. xietaTransf).  All output coefficients are in the
 *    orthonormal Dubiner basis of that frame: basis function 0 is the
 *    constant 1, functions 1..d are linear, ordered by total degree, then by
 *    the collapsed-coordinate indices p descending and q descending; they are
 *    orthonormal w.r.t. (1/|T_E|) times the integral over the unit simplex.
 *  - Periodic boxes use the minimum-image convention per periodic axis.
 *  - Device arrays are structure-of-arrays with the cell index fastest:
 *    q[v][i] (n_vars x n_cells) and coeffs[v][l][i] (n_vars x n_basis x n_cells).
 */
#ifndef CWENO_H
#define CWENO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CWENO_ABI_VERSION 1

typedef enum {
  CWENO_OK = 0,
  CWENO_E_ARG = -1,       /* invalid argument (NULL pointer, bad size, unsupported combination) */
  CWENO_E_MESH = -2,      /* degenerate cell, face shared by > 2 cells, vertex id out of range   */
  CWENO_E_STENCIL = -3,   /* a central stencil cannot be filled                                   */
  CWENO_E_RANK = -4,      /* rank-deficient least-squares system                                  */
  CWENO_E_PERIODIC = -5,  /* a stencil reaches too far across a periodic box (mesh too coarse)    */
  CWENO_E_NOMEM = -6,     /* host or device allocation failed                                     */
  CWENO_E_BUDGET = -7,    /* request exceeds a memory budget                                      */
  CWENO_E_HIP = -8,       /* a HIP runtime call failed                                            */
  CWENO_E_BUSY = -9,      /* resource in use                                                      */
  CWENO_E_CANCELLED = -10 /* request cancelled                                                    */
} cweno_status;

typedef enum {
  CWENO_F64 = 0,  /* double precision */
  CWENO_F32 = 1   /* single precision */
} cweno_dtype;

/* Which precisions of the per-cell operators a mesh keeps resident. */
typedef enum {
  CWENO_OPS_F64 = 0,
  CWENO_OPS_F32 = 1,
  CWENO_OPS_BOTH = 2,
  CWENO_OPS_NONE = 3   /* no stored operators (a moving mesh: see cweno_reconstruct_moving) */
} cweno_ops;

typedef enum {
  /* Sec. 2.1: sector s holds the cell and the nearest cells whose barycentre
   * lies in the open cone with apex at vertex s spanned by the edges towards
   * the other vertices (the cone through the face opposite vertex s). */
  CWENO_SECTOR_CONE = 0,
  /* Sector s = the cell and its face neighbours except the one across the
   * face opposite vertex s (exactly d+1 cells). */
  CWENO_SECTOR_FACE = 1
} cweno_sector_rule;

/* Option flags. */
#define CWENO_FLAG_HOST_ONLY 1u       /* build tables/operators on the host only; no device upload */
#define CWENO_FLAG_SIGMA0_POPT 2u     /* indicator of the central polynomial from P_opt, not P_0   */
#define CWENO_FLAG_LINEAR_WEIGHTS 4u  /* diagnostic: omega := lambda (w = P_opt)                   */
#define CWENO_FLAG_MOVING 8u          /* keep connectivity and stencils on the device for
                                         cweno_reconstruct_moving                                */
#define CWENO_FLAG_WENO 16u           /* the classical unstructured WENO scheme instead of CWENO
                                         (see cweno_mesh_weno_tables)                            */
#define CWENO_FLAG_DEVICE_OPERATORS 32u /* build the per-cell operators on the GPU (FP64) from the
                                         host's stencils, in the same stored layout; central
                                         stencils of at most 65 cells; not host-only, not WENO  */

/* Reconstruction options.  A zero-initialised struct gives the defaults. */
typedef struct {
  double periodic[3];      /* period per axis; 0 = not periodic                                  */
  double stencil_factor;   /* central stencil n_e = ceil(f * n_basis); 0 -> f = d (Sec. 2.1)   */
  double lambda0;          /* central linear weight in (0,1); 0 -> 0.95; negative -> the paper's
                              pair (1e5 central, 1 per sector, Sec. 2.1) normalised to sum 1.
                              Each sector gets (1 - lambda0)/(d+1).                              */
  double eps;              /* eps of the nonlinear weights; 0 -> 1e-14 (Sec. 2.1)              */
  int r;                   /* exponent r of the nonlinear weights; 0 -> 4 (Sec. 2.1)            */
  int ops;                 /* cweno_ops: operator precisions kept on the device; default F64    */
  int sector_rule;         /* cweno_sector_rule                                                  */
  unsigned flags;          /* CWENO_FLAG_*                                                       */
} cweno_options;

typedef struct cweno_mesh cweno_mesh;

/*
 * cweno_mesh_create -- register a mesh and precompute its reconstruction
 * operators (Sec. 2.1: stencils and inverted least-squares matrices are
 * computed once and stored for fixed meshes).
 *
 *  dim          2 (triangles) or 3 (tetrahedra)
 *  n_vertices   number of vertices (> 0)
 *  vertices     host, [n_vertices][dim] doubles; copied
 *  n_cells      number of cells (> 0, < 2^31)
 *  cells        host, [n_cells][dim+1] int32 vertex ids, 0-based; copied.  The
 *               order of each row fixes the cell's reference frame.
 *  degree       polynomial degree M, 1..4
 *  opt          options (NULL = defaults)
 *  hip_stream   stream for the device upload (NULL = default); the call
 *               synchronises it before returning
 *  out          receives the new mesh; owned by the caller, free with
 *               cweno_mesh_destroy
 *
 * Steps (host, FP64, multithreaded): minimum-image geometry, face adjacency,
 * central and sectorial stencils (Sec. 2.1, eq. stencil; breadth-first rings
 * of face neighbours ordered by squared barycentre distance, ties by lower
 * index), stencil averages of the basis in each cell's reference frame
 * (Gaussian quadrature), the least-squares pseudo-inverse for P_opt (eq.
 * CWENO:Popt, reduced exactly to an unconstrained problem on differences
 * because the basis has zero mean: p_0 = Q_i, p_{1..} = pinv(A') dQ), the
 * inverses of the sectorial P1 systems (eq. CWENO:Ps), and the universal
 * oscillation matrix Sigma.  A sector that cannot be filled or whose system
 * has condition number above 1e10 is dropped (its linear weight becomes 0,
 * the others are renormalised).
 *
 * Errors: CWENO_E_ARG, CWENO_E_MESH, CWENO_E_STENCIL, CWENO_E_RANK,
 * CWENO_E_PERIODIC, CWENO_E_NOMEM, CWENO_E_HIP.  On error *out is NULL.
 */
cweno_status cweno_mesh_create(int dim, int64_t n_vertices, const double* vertices,
                               int64_t n_cells, const int32_t* cells, int degree,
                               const cweno_options* opt, void* hip_stream, cweno_mesh** out);

/* Release a mesh and its device memory.  NULL is accepted.  The caller must
 * ensure no reconstruction on it is still running. */
cweno_status cweno_mesh_destroy(cweno_mesh* mesh);

/*
 * cweno_mesh_info -- sizes of a mesh.  Any output pointer may be NULL.
 *  n_cells       number of cells
 *  n_basis       basis size n_basis(M, d) = (1/d!) prod_{l=1..d} (M + l) (eq. cwenoM)
 *  n_e           central stencil size (cell included)
 *  gather_len    per-cell gather list length: n_e - 1 plus the mesh-wide maximum
 *                number of sector cells outside the central stencil
 *  device_bytes  bytes of device memory held by the mesh
 *  n_dropped     number of dropped sectors over the whole mesh
 */
cweno_status cweno_mesh_info(const cweno_mesh* mesh, int64_t* n_cells, int* n_basis, int* n_e,
                             int* gather_len, int64_t* device_bytes, int64_t* n_dropped);

/*
 * cweno_mesh_tables -- host copies of the integer tables (any pointer may be NULL).
 *  face_nbr  [n_cells][d+1]: the cell across the face opposite local vertex k, -1 = boundary
 *  stencil   [n_cells][n_e]: central stencil, the cell itself first (Sec. 2.1, j(1) = i)
 *  sectors   [n_cells][d+1][d+1]: sector s, the cell itself first; a dropped sector is a row of -1
 */
cweno_status cweno_mesh_tables(const cweno_mesh* mesh, int32_t* face_nbr, int32_t* stencil,
                               int32_t* sectors);

/*
 * cweno_mesh_operators -- host copies of the FP64 per-cell operators for one
 * cell (any pointer may be NULL).
 *  pinv   [(n_basis-1)][(n_e-1)]: P_opt coefficients 1.. = pinv * (Q_stencil[1..] - Q_i)
 *  binv   [d+1][d][d]: sector s linear coefficients 1..d = binv_s * (Q_sector[1..] - Q_i)
 *  sigma  [(n_basis-1)][(n_basis-1)]: oscillation matrix without the constant row/column
 */
cweno_status cweno_mesh_operators(const cweno_mesh* mesh, int64_t cell, double* pinv, double* binv,
                                  double* sigma);

/*
 * cweno_reconstruct -- the reconstruction of Sec. 2.1 for every cell and
 * variable of a mesh: (a) P_opt from the stored pseudo-inverse (eq.
 * CWENO:Popt), (b) the d+1 sectorial P1 polynomials (eq. CWENO:Ps), (c)
 * P_0 = (P_opt - sum_s lambda_s P_s)/lambda_0 (eq. CWENO:P0), (d) the
 * oscillation indicators sigma_s = p_s^T Sigma p_s, (e) the nonlinear weights
 * omega_s = lambda_s/(sigma_s+eps)^r normalised (eqs. weights, weights2) and
 * the blend w = sum_s omega_s P_s (eq. CWENO:Prec).
 *
 *  n_vars      number of variables (>= 1)
 *  dtype       precision of q, coeffs, sigma, omega and of the arithmetic;
 *              the mesh must hold operators of that precision
 *  q           device, [n_vars][n_cells] cell averages
 *  coeffs      device, [n_vars][n_basis][n_cells] output; coeffs[v][0][i] is a
 *              bitwise copy of q[v][i] (conservation)
 *  sigma       optional device output [n_vars][d+2][n_cells] (index 0 = central), or NULL
 *  omega       optional device output [n_vars][d+2][n_cells], or NULL
 *  hip_stream  stream to launch on (NULL = default)
 *
 * Asynchronous: it enqueues kernels and returns; it neither allocates nor
 * synchronises.  Buffers are owned by the caller and must stay valid until
 * the stream has executed the work.  The four buffers must not overlap.
 * Errors: CWENO_E_ARG (bad sizes, host-only mesh, missing operator precision,
 * overlapping buffers), CWENO_E_HIP (launch failure).
 */
cweno_status cweno_reconstruct(const cweno_mesh* mesh, int n_vars, cweno_dtype dtype,
                               const void* q, void* coeffs, void* sigma, void* omega,
                               void* hip_stream);

/*
 * cweno_reconstruct_moving -- the same reconstruction on a moving mesh: the
 * per-cell operators are rebuilt on the device from this call's vertex
 * positions instead of being read from memory (on an ALE mesh the
 * reconstruction matrices change with the geometry at every step, Sec. 2.1).
 *
 * The connectivity, the central and sectorial stencils and each cell's
 * reference frame (its vertex order) are those fixed at cweno_mesh_create;
 * only the vertex positions change.  Per cell and call the kernel computes,
 * in FP64: the cell's reference map from the moved vertices (minimum image
 * across periodic axes), the averages of psi_1 .. psi_{n_basis-1} over every
 * stencil cell in that frame (Grundmann-Moller quadrature exact to degree M),
 * the least-squares solve of eq. CWENO:Popt by Householder QR of the column-
 * scaled matrix, the sectorial systems of eq. CWENO:Ps from the linear basis
 * functions at the sector cells' barycentres (a sector whose system has
 * 2-norm condition number above 1e10 is dropped for this call), and then
 * P_0, the indicators, the weights and the blend exactly as
 * cweno_reconstruct does.  Nothing is stored between calls.
 *
 *  mesh      created with CWENO_FLAG_MOVING (any ops, CWENO_OPS_NONE keeps
 *            no stored operators at all); its central stencil may hold at
 *            most 129 cells; the work mapping is cweno_mesh_moving_shape's
 *  vertices  device, [n_vertices][dim] doubles: this call's positions
 *  n_vars, dtype, q, coeffs, sigma, omega
 *            as for cweno_reconstruct (FP32 averages and coefficients are
 *            converted to and from FP64 around the arithmetic; coefficient 0
 *            is the cell's own average, bit for bit)
 *  fault     optional device int: the kernel ORs 1 into it for a cell whose
 *            moved vertices give a singular reference map and 2 for a zero
 *            column or a rank-deficient least-squares system (R diagonal at
 *            or below 1e-12 of its largest entry); such a cell's outputs are
 *            not meaningful.  The caller clears it.  NULL: no report.
 *  hip_stream  stream of the launch (NULL = default); asynchronous
 *
 * No buffer may overlap another.  Errors: CWENO_E_ARG (bad arguments, a mesh
 * without CWENO_FLAG_MOVING, a stencil too large), CWENO_E_HIP.
 */
cweno_status cweno_reconstruct_moving(const cweno_mesh* mesh, const double* vertices, int n_vars,
                                      cweno_dtype dtype, const void* q, void* coeffs, void* sigma,
                                      void* omega, int* fault, void* hip_stream);

/*
 * cweno_mesh_set_moving_shape / cweno_mesh_moving_shape -- the work mapping
 * of cweno_reconstruct_moving (no effect on its results beyond rounding).
 * A segment of seg lanes (8, 16, 32 or 64) reconstructs one cell, each lane
 * holding rpl rows (1..4) of the cell's least-squares matrix; besides those,
 * seg = 4 with rpl = 5 is built for 2-D degree 3 and seg = 8 with rpl = 8 for
 * 3-D degree 3 (both the defaults there); narrower
 * segments need fewer exchange stages per sum over the rows and serve more
 * cells per wave.  By default the narrowest instantiated shape whose seg * rpl
 * row slots hold the central stencil (besides the cell) is used.
 *
 *  set:  seg = rpl = 0 restores the default; otherwise the shape must be
 *        instantiated for the mesh's (dim, degree) and hold its stencil.
 *        Not while another call uses the mesh.
 *  get:  seg, rpl (host ints) receive the shape the next call uses.
 *
 * Errors: CWENO_E_ARG (NULL pointers, a mesh without CWENO_FLAG_MOVING, a
 * shape that is not instantiated or too small for the stencil).
 */
cweno_status cweno_mesh_set_moving_shape(cweno_mesh* mesh, int seg, int rpl);
cweno_status cweno_mesh_moving_shape(const cweno_mesh* mesh, int* seg, int* rpl);

/*
 * Point values of the reconstruction (the predictor and the fluxes use the
 * reconstruction polynomial at quadrature points of each cell and of its
 * faces, Sec. 2.2-2.3).
 *
 * cweno_points_create   register a point set: n_points reference coordinates
 *                       (host, [n_points][dim] doubles; e.g. face or volume
 *                       quadrature points on the reference simplex), the same
 *                       relative place in every cell since every cell's
 *                       coefficients live in its own reference frame.  The
 *                       basis values phi[q][l] = psi_l(xi_q) (the library's
 *                       basis order) are computed once on the host in FP64
 *                       and kept on the current device in FP64 and FP32.
 *                       1 <= n_points <= 4096, degree 1..4.
 * cweno_points_basis    host copy of phi, [n_points][n_basis] (for tests)
 * cweno_points_destroy  release it (NULL accepted)
 * cweno_evaluate        values[v][q][i] = sum_l phi[q][l] coeffs[v][l][i] for
 *                       every cell i of the mesh: coeffs as written by
 *                       cweno_reconstruct (device, [n_vars][n_basis][n_cells]),
 *                       values device [n_vars][n_points][n_cells], both of
 *                       dtype; asynchronous on hip_stream; the point set must
 *                       have the mesh's dimension and degree; the buffers must
 *                       not overlap.  Errors: CWENO_E_ARG, CWENO_E_HIP.
 * cweno_reconstruct_points  cweno_reconstruct and cweno_evaluate in one pass:
 *                       the reconstruction kernel writes the polynomial's
 *                       values at the point set (values [n_vars][n_points]
 *                       [n_cells], dtype) instead of its coefficients, with
 *                       the same bits as the two calls in sequence.  Needs a
 *                       CWENO mesh with operators of dtype whose block halos
 *                       fit in LDS; n_points * n_cells values of one variable
 *                       below 4 GiB; q and values must not overlap.
 */
typedef struct cweno_points cweno_points;
cweno_status cweno_points_create(int dim, int degree, int n_points, const double* ref_points, cweno_points** out);
cweno_status cweno_points_basis(const cweno_points* points, double* phi);
cweno_status cweno_points_destroy(cweno_points* points);
cweno_status cweno_evaluate(const cweno_mesh* mesh, const cweno_points* points, int n_vars, cweno_dtype dtype,
                            const void* coeffs, void* values, void* hip_stream);
cweno_status cweno_reconstruct_points(const cweno_mesh* mesh, const cweno_points* points, int n_vars,
                                      cweno_dtype dtype, const void* q, void* values, void* hip_stream);

/*
 * Classical unstructured WENO (CWENO_FLAG_WENO at cweno_mesh_create): the
 * scheme the paper compares CWENO with in its efficiency discussion (Sec. 4),
 * built on the same geometry, quadrature and least squares.  n_s = 1 + 2(d+1)
 * stencils of n_e cells each: the central stencil, d+1 forward sectors (the
 * CWENO cones, filled to n_e cells) and d+1 reverse sectors (the opposite cone
 * at each vertex: every barycentric coordinate but the s-th below -1e-12);
 * each gives a degree-M polynomial by the constrained least squares of eq.
 * CWENO:Popt on its own stencil; indicators with the same Sigma; linear
 * weights lambda0 (central) and (1 - lambda0)/(2(d+1)) per sector (lambda0 < 0:
 * 1e5 against 1 per sector, normalised); omega~ = lambda/(sigma+eps)^r,
 * w = sum omega~ P / sum omega~.  An unfillable stencil is dropped.  Such a
 * mesh keeps FP64 operators only (ops must be CWENO_OPS_F64; no moving form,
 * no CWENO-only flags); cweno_reconstruct runs the WENO kernel (FP64, sigma and
 * omega must be NULL); it cannot join a batch or a server.  Creation fails
 * with CWENO_E_ARG if the stencils of 64 consecutive cells reference more than
 * 8192 distinct cells (the kernel stages that halo in LDS); a reconstruction
 * takes as many variables per pass as the largest such halo leaves room for.
 *
 * cweno_mesh_weno_tables  *n_stencils = n_s; stencils (may be NULL) receives
 *                         the host table [n_cells][n_s][n_e] int32 (the cell
 *                         first; a row of -1 for an unfillable stencil)
 */
cweno_status cweno_mesh_weno_tables(const cweno_mesh* mesh, int* n_stencils, int32_t* stencils);

/*
 * Kernel variants and their autotuner.
 *
 * The reconstruction kernel exists in several variants (cweno_num_variants()).
 * Kind 0 gathers the neighbour averages of each cell's stencil from global
 * memory; kind 1 first copies, per workgroup of 256 consecutive cells, the
 * averages of every cell their stencils reference (the block's halo, listed
 * by the library at cweno_mesh_create) into LDS and reads the stencils from
 * there.  Both walk the stencil in chunks of KC entries.  All variants
 * compute the same values (the per-lane sums run over the stencil in the same
 * order); they differ only in speed.  Kind 1 is available only when every
 * block's halo fits in LDS.  A mesh keeps one variant per (precision,
 * variable block); variables are processed in blocks of at most 9 (the block
 * sizes instantiated for the mesh's degree and dimension), each block reading
 * the operators once.
 *
 * cweno_mesh_set_variant  choose variant `variant` for blocks of `vb` variables
 *                         (CWENO_E_ARG if that combination is not instantiated)
 * cweno_mesh_get_variant  report the current choice (variant index, kind, KC)
 * cweno_mesh_tune         time every instantiated variant for each block that a
 *                         cweno_reconstruct of n_vars variables would launch,
 *                         using the caller's device buffers q [n_vars][n_cells]
 *                         and coeffs [n_vars][n_basis][n_cells] (coeffs is
 *                         overwritten), `repeats` timed launches per variant on
 *                         hip_stream, and keep the fastest.  Blocking: it
 *                         synchronises the stream.  *best_ms (may be NULL)
 *                         receives the tuned time of one full reconstruction.
 */
int cweno_num_variants(void);
cweno_status cweno_mesh_set_variant(cweno_mesh* mesh, cweno_dtype dtype, int vb, int variant);
cweno_status cweno_mesh_get_variant(const cweno_mesh* mesh, cweno_dtype dtype, int vb, int* variant, int* kind,
                                    int* kc);
cweno_status cweno_mesh_tune(cweno_mesh* mesh, int n_vars, cweno_dtype dtype, const void* q, void* coeffs,
                             int repeats, void* hip_stream, double* best_ms);

/*
 * Batched reconstruction: many meshes in one graph launch (persistent kernels).
 *
 * cweno_batch_create  registers `n` device meshes (each holding operators of
 *                     `dtype`), mesh i to be reconstructed with n_vars[i]
 *                     variables per run.  The meshes' variable blocks are
 *                     grouped by (dimension, degree, block size); each group
 *                     runs as one persistent LDS-halo kernel over a work list
 *                     of (mesh, block of 256 cells) items.  An autotuner times
 *                     every halo variant and grid size per group on scratch
 *                     buffers (zero averages) and keeps the fastest; with a
 *                     non-NULL tune_cache_path the choices are read from and
 *                     appended to that text file (one line per group).  The
 *                     groups are then captured into one HIP graph, one parallel
 *                     branch per group.  Blocking (it synchronises hip_stream).
 *                     The meshes must outlive the batch and must not be re-tuned
 *                     meanwhile.  Errors: CWENO_E_ARG (NULL or host-only mesh,
 *                     missing precision, a mesh whose block halos do not fit in
 *                     LDS, sizes beyond 32-bit offsets), CWENO_E_NOMEM,
 *                     CWENO_E_HIP.
 * cweno_batch_run     q[i] ([n_vars[i]][n_cells_i]) and coeffs[i]
 *                     ([n_vars[i]][n_basis_i][n_cells_i]) are device buffers of
 *                     mesh i, as for cweno_reconstruct.  Asynchronous on
 *                     hip_stream: one copy of the kernel-parameter table (from
 *                     pinned host memory) and one graph launch; runs of one batch
 *                     on different streams are serialised.  It does not allocate.
 * cweno_batch_info    number of groups, of work items, and the summed tuned time
 *                     of the group kernels in ms (any pointer may be NULL).
 * cweno_batch_group   group g: dimension, degree, variable block, entries, work
 *                     items, chosen variant and grid, tuned time in ms.
 */
typedef struct cweno_batch cweno_batch;
cweno_status cweno_batch_create(int n, cweno_mesh* const* meshes, const int* n_vars, cweno_dtype dtype,
                                const char* tune_cache_path, void* hip_stream, cweno_batch** out);
cweno_status cweno_batch_run(cweno_batch* batch, const void* const* q, void* const* coeffs, void* hip_stream);
cweno_status cweno_batch_info(const cweno_batch* batch, int* n_groups, int64_t* n_items, double* tuned_ms);
cweno_status cweno_batch_group(const cweno_batch* batch, int g, int* dim, int* degree, int* vb, int* n_entries,
                               int* n_items, int* variant, int* grid, double* ms);
cweno_status cweno_batch_destroy(cweno_batch* batch);

/*
 * Batched reconstruction that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the reconstructions of cweno_batch_create
 * plus cweno_batch_run in one call, without a batch object, a tuner or a graph.
 *
 * n meshes (device meshes holding operators of `dtype`, on the current
 * device); mesh i is reconstructed from q[i] ([n_vars[i]][n_cells_i]) into
 * coeffs[i] ([n_vars[i]][n_basis_i][n_cells_i]), device buffers as for
 * cweno_reconstruct, with the same bits.  The meshes' variable blocks are
 * grouped by (dimension, degree, block size) and each group runs as one launch
 * of the batched LDS-halo kernel.  Its launch table and work list live in a
 * static device array of 512 KiB + 256 table entries that each GPU holds for
 * the life of the process (filled from a static host stage with host-to-device
 * copies on hip_stream); the call makes no hipMalloc, hipFree or other
 * allocating call.  Limits: at most 256 variable blocks (a block holds up to 9,
 * 5 or fewer variables depending on the basis) and 65,536 blocks of 256 cells
 * over all meshes, else CWENO_E_ARG and nothing runs.  Every mesh's block
 * halos must fit in LDS (CWENO_E_ARG otherwise).  Asynchronous on hip_stream;
 * it may wait for the host-to-device copy of the previous call.  All calls on
 * one GPU share the device array: calls on different streams that are not
 * ordered with each other race and must not overlap.
 */
cweno_status cweno_batch_run_noalloc(int n, const cweno_mesh* const* meshes, const int* n_vars, cweno_dtype dtype,
                                     const void* const* q, void* const* coeffs, void* hip_stream);

/*
 * Serving: registered meshes, HBM residency under a budget, requests batched
 * as they arrive (continuous batching).
 *
 * cweno_server_create    an HBM arena of hbm_budget_bytes is allocated now (the
 *                        serving loop never allocates or frees device memory);
 *                        operators are kept in precision op_dtype; at most
 *                        max_inflight launches (1..256) run at once, spread
 *                        over n_streams compute streams (1..16).  Each launch
 *                        carries the requests queued when it starts, up to
 *                        64 (cweno_server_set_batch) and what one launch
 *                        table holds (512 variable blocks, 65,536 blocks of
 *                        256 cells); a request too large for the table, or
 *                        whose block halos do not fit in LDS, runs alone.
 *                        A scheduler thread and a completion thread start here.
 * cweno_server_register  host precompute of a mesh (arguments as for
 *                        cweno_mesh_create; opt->ops and HOST_ONLY are set by
 *                        the server) and one host image of its whole device
 *                        layout (pinned memory up to the pinned limit,
 *                        pageable beyond it).  *mesh_id receives its id.
 *                        CWENO_E_BUDGET if the image alone exceeds the budget.
 * cweno_server_register_mesh  the same from a mesh built with CWENO_FLAG_HOST_ONLY
 *                        (its precompute is reused; the caller keeps ownership
 *                        of host_mesh, which may be destroyed afterwards).
 * cweno_server_mesh_info cells, basis size, image bytes, currently resident.
 * cweno_server_submit    non-blocking: queues a reconstruction of mesh mesh_id
 *                        (q, coeffs: device buffers as for cweno_reconstruct,
 *                        in the server's precision, valid until the request is
 *                        done; the server's streams do not wait for the
 *                        caller's, so q must already hold its values) and
 *                        returns a ticket.  Requests are admitted in
 *                        submission order; a mesh that is not resident is
 *                        uploaded into the arena, evicting the least recently
 *                        used meshes that no running request uses.  Results
 *                        are the same bits as cweno_reconstruct's, alone or
 *                        batched with other requests.
 * cweno_server_poll      *done = 1 once the request has finished (or was
 *                        cancelled: CWENO_E_CANCELLED; or failed: CWENO_E_HIP).
 * cweno_server_wait      blocks until the request finishes or timeout_s passes
 *                        (timeout_s < 0: no limit; CWENO_E_BUSY on timeout).
 *                        Once poll or wait has reported a final state (done,
 *                        cancelled, failed), the ticket is released: later
 *                        calls with it return CWENO_E_ARG (unknown ticket).
 * cweno_server_cancel    removes a request that has not started
 *                        (CWENO_E_BUSY if it is running or finished).
 * cweno_server_stats     latency quantiles in seconds (completion seen by the
 *                        host minus submission), completed requests, evictions,
 *                        uploads and uploaded bytes since creation or the last
 *                        cweno_server_reset_stats.  Any pointer may be NULL.
 * cweno_server_set_batch requests one launch may carry (1..512; 1 = every
 *                        request launched on its own).
 * cweno_server_set_pinned_limit  bytes of mesh images registered from now on
 *                        that may be kept in pinned host memory (default
 *                        32 GiB); images beyond it are pageable (slower
 *                        uploads).  Pinned memory is a limited resource of the
 *                        host, which the runtime's own pageable copies need too.
 * cweno_server_launch_stats  launches started, requests that shared a launch
 *                        with others, the most requests in one launch (since
 *                        creation or the last reset), and the tickets the
 *                        server still holds (not yet reported final).
 * cweno_server_pause     paused != 0 holds admission (submitted requests stay
 *                        queued and can be cancelled); 0 resumes it.
 * cweno_server_destroy   cancels queued requests, waits for running ones.
 */
typedef struct cweno_server cweno_server;
cweno_status cweno_server_create(int64_t hbm_budget_bytes, cweno_dtype op_dtype, int max_inflight, int n_streams,
                                 cweno_server** out);
cweno_status cweno_server_register(cweno_server* server, int dim, int64_t n_vertices, const double* vertices,
                                   int64_t n_cells, const int32_t* cells, int degree, const cweno_options* opt,
                                   int64_t* mesh_id);
cweno_status cweno_server_register_mesh(cweno_server* server, const cweno_mesh* host_mesh, int64_t* mesh_id);
cweno_status cweno_server_mesh_info(cweno_server* server, int64_t mesh_id, int64_t* n_cells, int* n_basis,
                                    int64_t* image_bytes, int* resident);
cweno_status cweno_server_submit(cweno_server* server, int64_t mesh_id, int n_vars, cweno_dtype dtype,
                                 const void* q, void* coeffs, int64_t* ticket);
cweno_status cweno_server_poll(cweno_server* server, int64_t ticket, int* done);
cweno_status cweno_server_wait(cweno_server* server, int64_t ticket, double timeout_s);
cweno_status cweno_server_cancel(cweno_server* server, int64_t ticket);
cweno_status cweno_server_stats(cweno_server* server, double* p50_s, double* p99_s, double* p999_s,
                                int64_t* completed, int64_t* evictions, int64_t* uploads, int64_t* upload_bytes);
cweno_status cweno_server_reset_stats(cweno_server* server);
cweno_status cweno_server_set_batch(cweno_server* server, int max_batch);
cweno_status cweno_server_set_pinned_limit(cweno_server* server, int64_t bytes);
cweno_status cweno_server_launch_stats(cweno_server* server, int64_t* launches, int64_t* shared_requests,
                                       int64_t* largest_launch, int64_t* tickets_held);
cweno_status cweno_server_pause(cweno_server* server, int paused);
cweno_status cweno_server_destroy(cweno_server* server);

const char* cweno_status_string(cweno_status status);
const char* cweno_last_error(void);
int cweno_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CWENO_H */
