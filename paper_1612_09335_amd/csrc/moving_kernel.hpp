// CWENO reconstruction on a moving mesh (gfx950): the per-cell operators of
// Sec. 2.1 are not read from memory but rebuilt inside the kernel from this
// call's vertex positions, for the mesh's fixed connectivity and stencils.
// On a moving (ALE) mesh the reconstruction matrices change with the geometry
// at every step (Sec. 2.1), so storing them buys nothing; this trades the
// operator stream for arithmetic.
//
// Work mapping.  A segment of SEG lanes (4, 8, 16, 32 or 64) owns one cell.  Lane t
// of the segment owns rows t, t + SEG, ... (RPL rows) of the cell's least-
// squares matrix A' (row k: stencil cell k+1).  Per cell:
//   1. every lane unwraps the cell's vertices (minimum image around vertex 0)
//      and inverts its reference map x = X0 + J xi;
//   2. each row lane places its stencil cell in that frame (translated by the
//      minimum-image offset of the barycentres) and integrates psi_1 .. psi_NL
//      over it with the Grundmann-Moller rule exact to degree M (eq.
//      xietaTransf: every integral in the reference coordinates of the cell);
//   3. columns are scaled to unit 2-norm and reduced by Householder
//      reflections; the sums over the segment are butterflies (DPP within
//      rows of 16 lanes, a swizzle across rows, lane reads across the halves
//      of the wave), so a narrower segment with more rows per lane needs
//      fewer exchange stages per sum and serves more cells per wave
//      instruction (a sum of R rows per lane over S lanes costs R + 3 log2 S
//      wave instructions for 64 / S cells).  Each reflector stays in the entries it eliminated;
//   4. one lane per sector evaluates the linear basis functions at the sector
//      cells' barycentres (the averages of a linear function), inverts the
//      d x d system (eq. CWENO:Ps) and drops the sector if its 2-norm
//      condition number, sigma_max(B) sigma_max(B^-1), exceeds 1e10;
//   5. per pass of VB variables, the differences dQ of the row cells are
//      reflected, R and Q^T dQ go to LDS, and one lane per variable solves
//      R x = Q^T dQ, undoes the column scaling (P_opt, eq. CWENO:Popt with
//      p_0 = Q_i), and forms the sector polynomials, P_0, the indicators, the
//      nonlinear weights and the blend (eqs. CWENO:P0, weights, CWENO:Prec).
// Everything is FP64; the averages and coefficients may be FP32 (converted on
// load and on store; coefficient 0 is the cell's own average, bit for bit).
//
// A singular reference map ORs 1 into *fault, a zero column or a rank-
// deficient R (a diagonal entry at or below 1e-12 of the largest) ORs 2; the
// outputs of such a cell are not meaningful.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "reconstruct_kernel.hpp"

namespace cweno {

// Variables reflected together (a pass): 2, 4, 5 or 9; at most 5 where the
// basis has more than 15 functions (the register budget of the 3-D M >= 3
// rows) and on 8-lane segments, 4 on 4-lane segments (one lane per variable
// forms the blend).
__host__ __device__ constexpr int move_vb_max(int D, int M, int SEG) {
  return SEG == 4 ? 4 : nbasis_c(M, D) - 1 <= 14 && SEG >= 9 ? 9 : 5;
}
__host__ __device__ constexpr int move_vb(int D, int M, int SEG, int nv) {
  return nv <= 2 ? 2 : SEG == 4 ? 4 : (nv <= 5 || move_vb_max(D, M, SEG) == 5) ? 5 : 9;
}
constexpr int kMoveThreads = 256;  // four waves per block

// Waves per SIMD the register allocation must leave room for.  The 3-D
// degree-3 kernels with one stencil row per lane need 200-218 registers on
// their own (two waves); bounded to 168 they run three waves with a few
// spills, which measured 9% faster.  With two rows per lane they fit two
// waves (254 registers, 4 spills); with four (16 lanes per cell) they take
// the accumulation registers as well and run one wave of four cells, which
// measured 7% faster than two waves of two cells.  The 3-D degree-4 kernels
// need all 256 and would spill heavily.  The 2-D kernels are held to three
// waves up to degree 3 and to two at degree 4 (on 8 lanes each would
// otherwise take a few registers more than that allows and lose a wave:
// measured 0.57 against 0.42 ms at degree 4); the others fit unbounded.  With
// five rows per lane (4-lane segments) the per-cell LDS records of a block
// allow two waves, and the registers are held to that.
__host__ __device__ constexpr int move_min_waves(int D, int M, int RPL) {
  return D == 3 ? (M == 3 ? (RPL == 1 ? 3 : RPL == 2 ? 2 : 1) : 1) : M <= 3 && RPL <= 4 ? 3 : 2;
}

template <typename T>
struct MParams {
  const double* V;        // [n_vertices][D] positions for this call
  const int32_t* C;       // [nc][D+1] vertex ids of each cell
  const int32_t* S0;      // [nc][n_e] central stencil, the cell first
  const int32_t* SS;      // [nc][D+1][D+1] sector stencils, the cell first; first entry < 0: not filled
  const uint8_t* SP;      // [nc][D+1][D] row of each sector cell in the central stencil (its position - 1), 255: not in it
  const T* q;             // [nv][nc]
  T* out;                 // [nv][NB][nc]
  T* sig;                 // optional [nv][D+2][nc]
  T* om;                  // optional [nv][D+2][nc]
  int* fault;             // optional
  // operator assembly (the VB = 0 form): the stored-operator layout, row stride Np;
  // a NULL pointer skips that array
  double* pinv64;
  float* pinv32;
  double* binv64;
  float* binv32;
  uint8_t* mask;
  int64_t Np;
  double box[3];          // period per axis, 0 = none
  double ibox[3];         // 1 / period per axis, 0 = none
  double lam[5];          // linear weights lambda_0 .. lambda_{D+1}
  double eps;
  int64_t nc;
  int n_e, nv, r, sigma0_popt, linear_w;
};

// f(std::integral_constant<int, I>) for I = 0 .. N-1, each call with a
// compile-time index (register arrays are then indexed statically even where
// the loop body is too large for the unroller).
template <int I, int N>
struct StaticFor {
  template <typename F>
  __device__ __forceinline__ static void run(F& f) {
    f(std::integral_constant<int, I>{});
    StaticFor<I + 1, N>::run(f);
  }
};
template <int N>
struct StaticFor<N, N> {
  template <typename F>
  __device__ __forceinline__ static void run(F&) {}
};

// ---------------------------------------------------------------- lane exchange

__device__ __forceinline__ uint32_t lo32(double x) { return (uint32_t)__builtin_bit_cast(uint64_t, x); }
__device__ __forceinline__ uint32_t hi32(double x) { return (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 32); }
__device__ __forceinline__ double mkd(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | (uint64_t)lo);
}

// DPP move of a double: every lane reads the lane selected by CTRL (a
// permutation within each row of 16 lanes, so no lane is out of range).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  return mkd((uint32_t)__builtin_amdgcn_mov_dpp((int)lo32(x), CTRL, 0xF, 0xF, false),
             (uint32_t)__builtin_amdgcn_mov_dpp((int)hi32(x), CTRL, 0xF, 0xF, false));
}
// As dpp_d, written only to the lanes of the banks (groups of 4 lanes within
// each row) set in BANKS; the other lanes keep old.
template <int CTRL, int BANKS>
__device__ __forceinline__ double dpp_upd_d(double old, double x) {
  return mkd((uint32_t)__builtin_amdgcn_update_dpp((int)lo32(old), (int)lo32(x), CTRL, 0xF, BANKS, false),
             (uint32_t)__builtin_amdgcn_update_dpp((int)hi32(old), (int)hi32(x), CTRL, 0xF, BANKS, false));
}
// Swizzle (bit-mask mode) of a double within each group of 32 lanes.
template <int PAT>
__device__ __forceinline__ double swz_d(double x) {
  return mkd((uint32_t)__builtin_amdgcn_ds_swizzle((int)lo32(x), PAT),
             (uint32_t)__builtin_amdgcn_ds_swizzle((int)hi32(x), PAT));
}
// Value of lane l (wave-uniform l).
__device__ __forceinline__ double rdl_d(double x, int l) {
  return mkd((uint32_t)__builtin_amdgcn_readlane((int)lo32(x), l),
             (uint32_t)__builtin_amdgcn_readlane((int)hi32(x), l));
}

constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane 7-l within each 8
constexpr int kDppMirror = 0x140;     // lane 15-l within each 16
constexpr int kSwzXor16 = 0x401F;     // and 0x1f, xor 0x10
constexpr int kDppRowShl4 = 0x104;    // lane l + 4 within each 16
constexpr int kDppRowShr4 = 0x114;    // lane l - 4 within each 16

// x[c] for first <= c < last := the sum of x[c] over the lanes of the segment,
// the same bits in every lane (each stage pairs every lane with one lane of
// the other half of its group, whose partial sum it then shares).  Every lane
// of the wave must be active.
template <int SEG, int N>
__device__ __forceinline__ void seg_sum(double (&x)[N], int first = 0, int last = N) {
  static_assert(SEG == 4 || SEG == 8 || SEG == 16 || SEG == 32 || SEG == 64, "segment of 4, 8, 16, 32 or 64 lanes");
#pragma unroll
  for (int c = 0; c < N; ++c)
    if (c >= first && c < last) x[c] += dpp_d<kDppXor1>(x[c]);
#pragma unroll
  for (int c = 0; c < N; ++c)
    if (c >= first && c < last) x[c] += dpp_d<kDppXor2>(x[c]);
  if constexpr (SEG >= 8) {
#pragma unroll
    for (int c = 0; c < N; ++c)
      if (c >= first && c < last) x[c] += dpp_d<kDppHalfMirror>(x[c]);
  }
  if constexpr (SEG >= 16) {
#pragma unroll
    for (int c = 0; c < N; ++c)
      if (c >= first && c < last) x[c] += dpp_d<kDppMirror>(x[c]);
  }
  if constexpr (SEG >= 32) {
#pragma unroll
    for (int c = 0; c < N; ++c)
      if (c >= first && c < last) x[c] += swz_d<kSwzXor16>(x[c]);
  }
  if constexpr (SEG == 64) {
#pragma unroll
    for (int c = 0; c < N; ++c)
      if (c >= first && c < last) x[c] = rdl_d(x[c], 0) + rdl_d(x[c], 32);
  }
}

// Value of x in lane SRC of this lane's segment.  A 4-lane segment is a quad
// (quad_perm).  A 16-lane segment is one DPP row: the row's lane SRC is
// broadcast to the row (row_newbcast).  An 8-lane segment is half a row: lane SRC % 4 of every quad goes to its quad
// (quad_perm), then the quad that holds lane SRC of the segment goes to the
// segment's other quad (a row shift by 4 written to that quad's banks only).
template <int SEG, int SRC>
__device__ __forceinline__ double seg_bcast(double x, int seg) {
  static_assert(SRC >= 0 && SRC < SEG, "lane of the segment");
  if constexpr (SEG == 4) {
    return dpp_d<SRC * 0x55>(x);
  } else if constexpr (SEG == 8) {
    const double a = dpp_d<(SRC % 4) * 0x55>(x);
    if constexpr (SRC < 4) return dpp_upd_d<kDppRowShr4, 0xA>(a, a);
    else return dpp_upd_d<kDppRowShl4, 0x5>(a, a);
  } else if constexpr (SEG == 16) {
    return dpp_d<0x150 + SRC>(x);
  } else if constexpr (SEG == 64) {
    return rdl_d(x, SRC);
  } else {
    const double a = rdl_d(x, SRC), b = rdl_d(x, SRC + 32);
    return seg ? b : a;
  }
}

// Orders the LDS accesses of the lanes of one wave: a wave-scope release
// fence, a wave barrier and an acquire fence.  Every per-cell LDS record is
// written and read by the lanes of its own segment, and a segment never spans
// two waves, so no workgroup barrier is needed (with one wave per SIMD, one
// would hold all four SIMDs of a workgroup to its slowest wave).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- small dense algebra

// 1/x for finite non-zero x whose reciprocal is a normal number (either sign):
// the refined hardware estimate, within an ulp or two of the quotient.
__device__ __forceinline__ double rcp_nz(double x) { return rcp_pos(x); }

// sqrt(x) for finite x >= 0 (0 for 0), within about an ulp: the hardware
// estimate y of 1/sqrt(x), one Goldschmidt step on g = x y, h = y / 2
// (r = 1/2 - g h; g += g r; h += h r), then two corrections g += (x - g^2) h.
__device__ __forceinline__ double sqrt_nn(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  g = fma(fma(-g, g, x), h, g);
  g = fma(fma(-g, g, x), h, g);
  return x > 0.0 ? g : 0.0;
}

// Minimum image of a difference d along an axis of period L (iL = 1/L; L = 0:
// not periodic).  The product by the reciprocal decides the same image as a
// quotient would except within rounding of half a period, which no stencil
// spans.
__device__ __forceinline__ double min_image_d(double d, double L, double iL) {
  return L != 0.0 ? d - L * floor(d * iL + 0.5) : d;
}

// Inverse of a small dense matrix (Gauss-Jordan, partial pivoting); false if
// a pivot vanishes.
template <int N>
__device__ __forceinline__ bool invert_small(const double (&A)[N][N], double (&Ai)[N][N]) {
  double W[N][2 * N];
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < 2 * N; ++c) W[r][c] = c < N ? A[r][c] : (c - N == r ? 1.0 : 0.0);
  bool ok = true;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    // pivot row brought to position c by conditional swaps (no dynamic indexing)
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      const bool sw = fabs(W[r][c]) > fabs(W[c][c]);
#pragma unroll
      for (int k = 0; k < 2 * N; ++k) {
        const double a = W[c][k], b = W[r][k];
        W[c][k] = sw ? b : a;
        W[r][k] = sw ? a : b;
      }
    }
    const double pv = W[c][c];
    ok = ok && pv != 0.0;
    const double ip = rcp_nz(pv);   // meaningless where pv = 0 (ok is then false)
#pragma unroll
    for (int k = 0; k < 2 * N; ++k) W[c][k] *= ip;
#pragma unroll
    for (int r = 0; r < N; ++r) {
      if (r == c) continue;
      const double f = W[r][c];
#pragma unroll
      for (int k = 0; k < 2 * N; ++k) W[r][k] = fma(-f, W[c][k], W[r][k]);
    }
  }
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) Ai[r][c] = W[r][N + c];
  return ok;
}

// Largest eigenvalue of B^T B (the squared largest singular value of B) in
// closed form: the larger root of the 2 x 2 characteristic polynomial, or the
// trigonometric solution of the symmetric 3 x 3 one (for the largest root
// neither loses relative accuracy).
template <int N>
__device__ __forceinline__ double sigma_max_sq(const double (&B)[N][N]) {
  double S[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(B[k][i], B[k][j], s);
      S[i][j] = s;
    }
  if constexpr (N == 2) {
    const double h = 0.5 * (S[0][0] - S[1][1]);
    return 0.5 * (S[0][0] + S[1][1]) + sqrt(fma(h, h, S[0][1] * S[0][1]));
  } else {
    static_assert(N == 3, "2 x 2 or 3 x 3");
    const double p1 = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2];
    const double q = (S[0][0] + S[1][1] + S[2][2]) / 3.0;
    if (!(p1 > 0.0)) return fmax(S[0][0], fmax(S[1][1], S[2][2]));
    const double a = S[0][0] - q, b = S[1][1] - q, c = S[2][2] - q;
    const double p = sqrt((a * a + b * b + c * c + 2.0 * p1) / 6.0);
    const double ip = 1.0 / p;
    const double x = a * ip, y = b * ip, z = c * ip, u = S[0][1] * ip, v = S[0][2] * ip, w = S[1][2] * ip;
    const double det = x * (y * z - w * w) - u * (u * z - w * v) + v * (u * w - y * v);
    const double r = fmin(1.0, fmax(-1.0, 0.5 * det));
    return q + 2.0 * p * cos(acos(r) / 3.0);
  }
}

// ---------------------------------------------------------------- basis

// Homogenised Jacobi values H[0..n] with parameter alpha at (u, v):
// H_n = v^n P_n^(alpha,0)(u/v) by the three-term recurrence multiplied through
// by powers of v; n and alpha are compile-time constants after unrolling.
template <int NMAX>
__device__ __forceinline__ void jac_h(int n, int alpha, double u, double v, double (&H)[NMAX + 1]) {
  H[0] = 1.0;
  if (n >= 1) H[1] = ((alpha + 2) * u + alpha * v) / 2.0;
  const double v2 = v * v;
#pragma unroll
  for (int k = 1; k < NMAX; ++k) {
    if (k >= n) break;
    const double a1 = 2.0 * (k + 1) * (k + alpha + 1) * (2.0 * k + alpha);
    const double c2 = (2.0 * k + alpha + 1) * alpha * alpha / a1;
    const double c3 = (2.0 * k + alpha) * (2.0 * k + alpha + 1) * (2.0 * k + alpha + 2) / a1;
    const double c4 = 2.0 * k * (k + alpha) * (2.0 * k + alpha + 2) / a1;
    H[k + 1] = (c3 * u + c2 * v) * H[k] - c4 * v2 * H[k - 1];
  }
}

// Position of psi_{p,q,r} in the library's order of the basis: total degree
// n = p + q + r, then p descending, then q descending (r = 0 in 2-D).
__host__ __device__ constexpr int basis_index(int D, int p, int q, int r) {
  const int n = p + q + r;
  int l = n == 0 ? 0 : nbasis_c(n - 1, D);
  if (D == 2) return l + (n - p);
  for (int pp = n; pp > p; --pp) l += n - pp + 1;
  return l + (n - p - q);
}

// Normalisation of psi_{p,q,r} (r = 0 in 2-D): the constant that makes the
// collapsed-coordinate product of Jacobi polynomials orthonormal,
// (1/|T_E|) int psi^2 = 1.
template <int D>
__device__ __forceinline__ double basis_norm(int p, int q, int r) {
  return D == 2 ? __builtin_sqrt((2.0 * p + 1.0) * (p + q + 1.0))
                : __builtin_sqrt((2.0 * p + 1.0) * (2.0 * p + 2.0 * q + 2.0) * (2.0 * p + 2.0 * q + 2.0 * r + 3.0) / 6.0);
}

// acc[l - 1] += w * psi_l(xi) / n_l for l = 1 .. NB-1, n_l the normalisation
// of psi_l (applied once to the sums by basis_normalise): the orthonormal
// collapsed-coordinate (Dubiner) basis evaluated factor by factor, so that no
// table of all values is held.
template <int D, int M>
__device__ __forceinline__ void basis_accumulate(const double (&xi)[D], double w, double (&acc)[nbasis_c(M, D) - 1]) {
  if constexpr (D == 2) {
    const double x = xi[0], y = xi[1];
    double F[M + 1];
    jac_h<M>(M, 0, 2.0 * x + y - 1.0, 1.0 - y, F);
#pragma unroll
    for (int p = 0; p <= M; ++p) {
      double G[M + 1];
      jac_h<M>(M - p, 2 * p + 1, 2.0 * y - 1.0, 1.0, G);
      const double wf = w * F[p];
#pragma unroll
      for (int q = 0; q <= M; ++q) {
        if (p + q == 0 || p + q > M) continue;
        const int l = basis_index(2, p, q, 0);
        acc[l - 1] = fma(wf, G[q], acc[l - 1]);
      }
    }
  } else {
    const double x = xi[0], y = xi[1], z = xi[2];
    double F[M + 1];
    jac_h<M>(M, 0, 2.0 * x + y + z - 1.0, 1.0 - y - z, F);
#pragma unroll
    for (int p = 0; p <= M; ++p) {
      double H[M + 1];
      jac_h<M>(M - p, 2 * p + 1, 2.0 * y + z - 1.0, 1.0 - z, H);
#pragma unroll
      for (int q = 0; q <= M; ++q) {
        if (p + q > M) continue;
        double K[M + 1];
        jac_h<M>(M - p - q, 2 * p + 2 * q + 2, 2.0 * z - 1.0, 1.0, K);
        const double wfh = w * F[p] * H[q];
#pragma unroll
        for (int r = 0; r <= M; ++r) {
          if (p + q + r == 0 || p + q + r > M) continue;
          const int l = basis_index(3, p, q, r);
          acc[l - 1] = fma(wfh, K[r], acc[l - 1]);
        }
      }
    }
  }
}

// acc[l - 1] *= n_l: the sums of basis_accumulate made sums of psi_l.
template <int D, int M>
__device__ __forceinline__ void basis_normalise(double (&acc)[nbasis_c(M, D) - 1]) {
#pragma unroll
  for (int p = 0; p <= M; ++p)
#pragma unroll
    for (int q = 0; q <= M; ++q)
#pragma unroll
      for (int r = 0; r <= (D == 3 ? M : 0); ++r) {
        if (p + q + r == 0 || p + q + r > M) continue;
        acc[basis_index(D, p, q, r) - 1] *= basis_norm<D>(p, q, r);
      }
}

// The d linear basis functions psi_1 .. psi_d at xi.
template <int D>
__device__ __forceinline__ void linear_basis(const double (&xi)[D], double (&out)[D]) {
  double acc[D];
#pragma unroll
  for (int l = 0; l < D; ++l) acc[l] = 0.0;
  basis_accumulate<D, 1>(xi, 1.0, acc);
  basis_normalise<D, 1>(acc);
#pragma unroll
  for (int l = 0; l < D; ++l) out[l] = acc[l];
}

// ---------------------------------------------------------------- quadrature

// The Grundmann-Moller rule on the D-simplex of degree 2s + 1, s = M / 2 (the
// smallest odd degree >= M), for averages: for i = 0 .. s and every
// beta in N^(D+1) with |beta| = s - i, the point with barycentric
// coordinates (2 beta_k + 1) / g, g = D + 2s + 1 - 2i, and weight
// D! (-1)^i 2^(-2s) g^(2s+1) / (i! (D + 2s + 1 - i)!) (Grundmann and Moller,
// SIAM J. Numer. Anal. 15, 1978; the weights sum to 1).  Built at compile
// time, so that the points and weights are immediates of the unrolled code.
__host__ __device__ constexpr int gm_points_c(int D, int M) {
  int n = 0;
  for (int i = 0; i <= M / 2; ++i) {
    const int m = M / 2 - i;   // compositions of m into D + 1 parts: C(m + D, D)
    int c = 1;
    for (int k = 1; k <= D; ++k) c = c * (m + k) / k;
    n += c;
  }
  return n;
}

template <int D, int M>
struct GMRule {
  static constexpr int NQ = gm_points_c(D, M);
  double lam[NQ][D + 1];
  double w[NQ];
  constexpr GMRule() : lam{}, w{} {
    const int s = M / 2;
    double fd = 1.0;
    for (int k = 2; k <= D; ++k) fd *= k;
    int q = 0;
    for (int i = 0; i <= s; ++i) {
      const int g = D + 2 * s + 1 - 2 * i, m = s - i;
      double c = (i % 2) ? -fd : fd;
      for (int k = 0; k < 2 * s; ++k) c *= 0.5;
      for (int k = 0; k < 2 * s + 1; ++k) c *= g;
      for (int k = 2; k <= i; ++k) c /= k;
      for (int k = 2; k <= D + 2 * s + 1 - i; ++k) c /= k;
      // every beta in [0, m]^(D+1) with |beta| = m, as the digits of t in base m + 1
      int span = 1;
      for (int k = 0; k <= D; ++k) span *= m + 1;
      for (int t = 0; t < span; ++t) {
        int b[D + 1] = {}, sum = 0, x = t;
        for (int k = 0; k <= D; ++k) {
          b[k] = x % (m + 1);
          x /= m + 1;
          sum += b[k];
        }
        if (sum != m) continue;
        for (int k = 0; k <= D; ++k) lam[q][k] = (2.0 * b[k] + 1.0) / g;
        w[q] = c;
        ++q;
      }
    }
  }
};

template <int D, int M>
struct GMTable {
  static constexpr GMRule<D, M> v{};
};

// ---------------------------------------------------------------- geometry

// Vertices X of a cell moved to their minimum images around vertex 0.
template <int D, typename T>
__device__ __forceinline__ void unwrap_vertices(const MParams<T>& p, double (&X)[D + 1][D]) {
#pragma unroll
  for (int v = 1; v <= D; ++v)
#pragma unroll
    for (int a = 0; a < D; ++a) X[v][a] = X[0][a] + min_image_d(X[v][a] - X[0][a], p.box[a], p.ibox[a]);
}

// Vertices of cell c, each moved to its minimum image around vertex 0.
template <int D, typename T>
__device__ __forceinline__ void cell_vertices(const MParams<T>& p, int64_t c, double (&X)[D + 1][D]) {
  int32_t id[D + 1];
#pragma unroll
  for (int v = 0; v <= D; ++v) id[v] = p.C[c * (D + 1) + v];
#pragma unroll
  for (int v = 0; v <= D; ++v)
#pragma unroll
    for (int a = 0; a < D; ++a) X[v][a] = p.V[(int64_t)id[v] * D + a];
  unwrap_vertices<D>(p, X);
}

template <int D>
__device__ __forceinline__ void barycentre(const double (&X)[D + 1][D], double (&c)[D]) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double s = X[0][a];
#pragma unroll
    for (int v = 1; v <= D; ++v) s = s + X[v][a];
    c[a] = s * (1.0 / (D + 1));
  }
}

// ---------------------------------------------------------------- kernel

template <int D, int M, int SEG, int RPL, int VB, typename T>
__global__ __launch_bounds__(kMoveThreads) __attribute__((amdgpu_waves_per_eu(move_min_waves(D, M, RPL))))
void moving_kernel(MParams<T> p) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NS = D + 1;
  constexpr int CPW = 64 / SEG;                          // cells per wave
  constexpr int CPB = (kMoveThreads / 64) * CPW;         // cells per block
  constexpr int CH = 8;                                  // column sums in flight
  static_assert(NL < SEG * RPL, "the rows of R lie in the segment's row slots");
  static_assert(VB <= SEG && NS <= SEG, "one lane per variable and per sector");
  // per-cell LDS record (doubles): P_opt of a pass of variables (or, when
  // assembling operators, the rows of R), column scales, diagonal of R,
  // reflector factors, sector inverses, each row cell's barycentre in the
  // cell's reference frame
  constexpr int OP = 0, OR = 0, OSC = OP + (VB > 0 ? VB * NL : NL * NL), ORD = OSC + NL, OTAU = ORD + NL,
                OBI = OTAU + NL, OXI = OBI + NS * D * D, OSZ = OXI + SEG * RPL * D;
  static_assert(VB > 0 || RPL == 1, "operator assembly keeps one row per lane");
  __shared__ double lds[CPB * OSZ];
  __shared__ int32_t ljs[CPB * NS * D];

  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const int seg = lane / SEG, sl = lane % SEG;
  const int cs = wave * CPW + seg;
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * CPB + cs;
  const bool valid = i < p.nc;
  const int64_t ic = valid ? i : p.nc - 1;
  double* const L = lds + cs * OSZ;
  int32_t* const LJ = ljs + cs * NS * D;
  const int NE1 = p.n_e - 1;
  const int64_t nc = p.nc;
  int fault = 0;

  // 1. the cell's own frame
  double X0[D], Jinv[D][D], ci[D];
  {
    double X[NS][D];
    cell_vertices<D>(p, ic, X);
    double J[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      X0[r] = X[0][r];
#pragma unroll
      for (int c = 0; c < D; ++c) J[r][c] = X[c + 1][r] - X[0][r];
    }
    if (!invert_small<D>(J, Jinv)) fault |= 1;
    barycentre<D>(X, ci);
  }

  // 2. rows of A': averages of psi_1 .. psi_NL over the stencil cells.  The
  // gathers of all the lane's rows go out level by level (stencil ids, vertex
  // ids, positions) before any row is integrated, so that the lane waits once
  // per level rather than once per level and row (a row slot past the
  // stencil gathers the cell itself).  With rules of up to 5 points the rows
  // are integrated without a branch and a slot past the stencil is zeroed
  // afterwards, so that the scheduler may interleave them; the larger rules
  // of M = 4 skip such a slot, one row at a time (interleaved, their rows
  // would not fit the registers).
  constexpr bool kRowBranch = GMRule<D, M>::NQ > 5;
  int row[RPL];
  bool rv[RPL];
  int32_t jr[RPL];
  double A[RPL][NL];
  double XR[RPL][NS][D];
  {
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      row[t] = sl + SEG * t;
      rv[t] = row[t] < NE1;
      jr[t] = rv[t] ? p.S0[ic * p.n_e + row[t] + 1] : (int32_t)ic;
    }
    int32_t vid[RPL][NS];
#pragma unroll
    for (int t = 0; t < RPL; ++t)
#pragma unroll
      for (int v = 0; v < NS; ++v) vid[t][v] = p.C[(int64_t)jr[t] * NS + v];
#pragma unroll
    for (int t = 0; t < RPL; ++t)
#pragma unroll
      for (int v = 0; v < NS; ++v)
#pragma unroll
        for (int a = 0; a < D; ++a) XR[t][v][a] = p.V[(int64_t)vid[t][v] * D + a];
  }
  auto row_t = [&](auto tc) {
    constexpr int t = decltype(tc)::value;
    double a[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) a[l] = 0.0;
    if (!kRowBranch || rv[t]) {
      double X[NS][D], cj[D], sh[D], Y[NS][D];
#pragma unroll
      for (int v = 0; v < NS; ++v)
#pragma unroll
        for (int b = 0; b < D; ++b) X[v][b] = XR[t][v][b];
      unwrap_vertices<D>(p, X);
      barycentre<D>(X, cj);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double dc = cj[a] - ci[a];
        sh[a] = min_image_d(dc, p.box[a], p.ibox[a]) - dc;
      }
      {   // the barycentre in the cell's frame, for the sector lanes
        double y[D];
#pragma unroll
        for (int b = 0; b < D; ++b) y[b] = ci[b] + min_image_d(cj[b] - ci[b], p.box[b], p.ibox[b]) - X0[b];
#pragma unroll
        for (int r = 0; r < D; ++r) {
          double t2 = 0.0;
#pragma unroll
          for (int b = 0; b < D; ++b) t2 = fma(Jinv[r][b], y[b], t2);
          L[OXI + row[t] * D + r] = t2;
        }
      }
#pragma unroll
      for (int v = 0; v < NS; ++v) {
        double y[D];
#pragma unroll
        for (int a = 0; a < D; ++a) y[a] = X[v][a] + sh[a] - X0[a];
#pragma unroll
        for (int r = 0; r < D; ++r) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < D; ++a) s = fma(Jinv[r][a], y[a], s);
          Y[v][r] = s;
        }
      }
      using GM = GMTable<D, M>;
      auto point = [&](int qq) {
        double xi[D];
#pragma unroll
        for (int r = 0; r < D; ++r) xi[r] = 0.0;
#pragma unroll
        for (int v = 0; v < NS; ++v)
#pragma unroll
          for (int r = 0; r < D; ++r) xi[r] = fma(GM::v.lam[qq][v], Y[v][r], xi[r]);
        basis_accumulate<D, M>(xi, GM::v.w[qq], a);
      };
      // rules of up to 10 points unrolled (their points become immediates);
      // the 15-point rule of 3-D M = 4 stays a loop, whose unrolled body
      // would spill to scratch memory
      if constexpr (GMRule<D, M>::NQ <= 10) {
#pragma unroll
        for (int qq = 0; qq < GMRule<D, M>::NQ; ++qq) point(qq);
      } else {
#pragma unroll 1
        for (int qq = 0; qq < GMRule<D, M>::NQ; ++qq) point(qq);
      }
      basis_normalise<D, M>(a);
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) A[t][l] = kRowBranch || rv[t] ? a[l] : 0.0;
  };
  StaticFor<0, RPL>::run(row_t);

  // the sector stencil of sector sl (its cells and their rows in the central
  // stencil), gathered here so that the latency overlaps the QR; lanes past
  // the sectors read sector 0's and do not use it
  int32_t ssr[NS];
  int spr[D];
  {
    const int64_t at = ic * NS + (sl < NS ? sl : 0);
#pragma unroll
    for (int k = 0; k < NS; ++k) ssr[k] = p.SS[at * NS + k];
#pragma unroll
    for (int a = 0; a < D; ++a) spr[a] = p.SP[at * D + a];
  }

  // 3a. unit column norms
  {
    double cn[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) s = fma(A[t][c], A[t][c], s);
      cn[c] = s;
    }
    seg_sum<SEG, NL>(cn, 0);
#pragma unroll
    for (int c = 0; c < NL; ++c) {
      const double s = sqrt_nn(cn[c]);
      fault |= s > 0.0 ? 0 : 2;
      const double is = rcp_pos(s);
#pragma unroll
      for (int t = 0; t < RPL; ++t) A[t][c] *= is;
      L[OSC + c] = s;   // every lane of the segment holds the same bits
    }
  }
  // 3b. Householder QR; reflector k replaces column k from row k down (the
  // steps and column chunks are expanded at compile time, so that A stays in
  // registers however large the unrolled body)
  auto qr_step = [&](auto kc) {
    constexpr int k = decltype(kc)::value;
    double x[RPL];
    double nn[1] = {0.0};
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      x[t] = row[t] >= k ? A[t][k] : 0.0;
      nn[0] = fma(x[t], x[t], nn[0]);
    }
    seg_sum<SEG, 1>(nn, 0);
    const double nrm = sqrt_nn(nn[0]);
    const double akk = seg_bcast<SEG, k % SEG>(A[k / SEG][k], seg);
    const double alpha = akk > 0.0 ? -nrm : nrm;
    const double vn2 = 2.0 * nrm * (nrm + fabs(akk));   // |x - alpha e_k|^2
    fault |= vn2 > 0.0 ? 0 : 2;
    const double tau = vn2 > 0.0 ? 2.0 * rcp_pos(vn2) : 0.0;
    double vk[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) vk[t] = row[t] == k ? akk - alpha : x[t];
    // the columns right of k, in chunks of CH reduced together
    auto chunk = [&](auto cc) {
      constexpr int c0 = decltype(cc)::value * CH;
      if constexpr (c0 + CH > k + 1) {
      double dot[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int c = c0 + u < NL ? c0 + u : NL - 1;
        double s = 0.0;
        if (c0 + u > k && c0 + u < NL) {
#pragma unroll
          for (int t = 0; t < RPL; ++t) s = fma(vk[t], A[t][c], s);
        }
        dot[u] = s;
      }
      seg_sum<SEG, CH>(dot, k + 1 - c0 > 0 ? k + 1 - c0 : 0, NL - c0 < CH ? NL - c0 : CH);
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int c = c0 + u < NL ? c0 + u : NL - 1;
        if (c0 + u > k && c0 + u < NL) {
          const double f = -tau * dot[u];
#pragma unroll
          for (int t = 0; t < RPL; ++t) A[t][c] = fma(f, vk[t], A[t][c]);
        }
      }
      }
    };
    StaticFor<0, (NL + CH - 1) / CH>::run(chunk);
#pragma unroll
    for (int t = 0; t < RPL; ++t)
      if (row[t] >= k) A[t][k] = vk[t];
    // the same bits in every lane of the segment: written without a branch,
    // so that nothing divides the steps for the scheduler
    L[ORD + k] = alpha;
    L[OTAU + k] = tau;
  };
  StaticFor<0, NL>::run(qr_step);

  wave_sync();   // the row cells' barycentres in LDS
  // 4. sectors: lane s of the segment builds and inverts sector s
  bool kept = false;
  if (sl < NS) {
    const int s = sl;
    double Bi[D][D];
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
      for (int a = 0; a < D; ++a) Bi[l][a] = 0.0;
    int32_t sj[D];
#pragma unroll
    for (int a = 0; a < D; ++a) sj[a] = (int32_t)ic;
    if (ssr[0] >= 0) {
      double B[D][D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        sj[a] = ssr[a + 1];
        double xi[D];
        const int pos = spr[a];
        if (pos != 255) {   // a central-stencil cell: its row lane left the barycentre in LDS
#pragma unroll
          for (int r = 0; r < D; ++r) xi[r] = L[OXI + pos * D + r];
        } else {
          double X[NS][D], cj[D], y[D];
          cell_vertices<D>(p, sj[a], X);
          barycentre<D>(X, cj);
#pragma unroll
          for (int b = 0; b < D; ++b) y[b] = ci[b] + min_image_d(cj[b] - ci[b], p.box[b], p.ibox[b]) - X0[b];
#pragma unroll
          for (int r = 0; r < D; ++r) {
            double t = 0.0;
#pragma unroll
            for (int b = 0; b < D; ++b) t = fma(Jinv[r][b], y[b], t);
            xi[r] = t;
          }
        }
        linear_basis<D>(xi, B[a]);
      }
      // 2-norm condition number k = sigma_max(B) sigma_max(B^-1), kept up to
      // 1e10.  The Frobenius product kF = |B|_F |B^-1|_F bounds it,
      // k <= kF <= d k, and decides unless kF lies in (1e10, d 1e10]; only
      // there are the largest singular values computed
      double Binv[D][D];
      bool keep = invert_small<D>(B, Binv);
      if (keep) {
        double fb = 0.0, fi = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l)
#pragma unroll
          for (int a = 0; a < D; ++a) {
            fb = fma(B[l][a], B[l][a], fb);
            fi = fma(Binv[l][a], Binv[l][a], fi);
          }
        const double kf2 = fb * fi;
        keep = kf2 <= 1e20;
        if (!keep && kf2 <= (double)(D * D) * 1e20) keep = sigma_max_sq<D>(B) * sigma_max_sq<D>(Binv) <= 1e20;
      }
      if (keep) {
        kept = true;
#pragma unroll
        for (int l = 0; l < D; ++l)
#pragma unroll
          for (int a = 0; a < D; ++a) Bi[l][a] = Binv[l][a];
      }
    }
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
      for (int a = 0; a < D; ++a) L[OBI + (s * D + l) * D + a] = Bi[l][a];
#pragma unroll
    for (int a = 0; a < D; ++a) LJ[s * D + a] = sj[a];
  }
  const unsigned kmask = (unsigned)(__ballot(kept) >> (seg * SEG)) & ((1u << NS) - 1u);
  wave_sync();

  // linear weights of the cell: dropped sectors get 0, the rest renormalised
  double lam[NS + 1];
  {
    double lsum = p.lam[0];
    lam[0] = p.lam[0];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      lam[s + 1] = ((kmask >> s) & 1u) ? p.lam[s + 1] : 0.0;
      lsum += lam[s + 1];
    }
    const double il = rcp_pos(lsum);
#pragma unroll
    for (int s = 0; s <= NS; ++s) lam[s] *= il;
  }
  const double inv_l0 = rcp_pos(lam[0]);

  if (sl == 0) {   // rank: every diagonal entry of R above 1e-12 of the largest
    double rmax = 0.0;
#pragma unroll
    for (int k = 0; k < NL; ++k) rmax = fmax(rmax, fabs(L[ORD + k]));
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (!(fabs(L[ORD + k]) > 1e-12 * rmax)) fault |= 2;
  }

  if constexpr (VB == 0) {
    // 5'. operator assembly: the pseudo-inverse D^-1 R^-1 Q1^T and the sector
    // inverses in the stored-operator layout (the same operators the host
    // builder writes).  Rows of R to LDS for every row lane's back substitution.
    if (row[0] < NL) {
#pragma unroll
      for (int c = 0; c < NL; ++c)
        if (c > row[0]) L[OR + row[0] * NL + c] = A[0][c];
    }
    // row r of Q1 = H_0 ... H_{NL-1} [I; 0]; column c changes only under H_k, k <= c
    double q1[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) q1[c] = row[0] == c ? 1.0 : 0.0;
    auto orth = [&](auto kc) {
      constexpr int k = NL - 1 - decltype(kc)::value;
      const double tau = L[OTAU + k];
      const double vk = row[0] >= k ? A[0][k] : 0.0;
      auto chunk = [&](auto cc) {
        constexpr int c0 = decltype(cc)::value * CH;
        if constexpr (c0 + CH > k) {
          double dot[CH];
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            const int c = c0 + u < NL ? c0 + u : NL - 1;
            dot[u] = (c0 + u >= k && c0 + u < NL) ? vk * q1[c] : 0.0;
          }
          seg_sum<SEG, CH>(dot, k - c0 > 0 ? k - c0 : 0, NL - c0 < CH ? NL - c0 : CH);
#pragma unroll
          for (int u = 0; u < CH; ++u) {
            const int c = c0 + u < NL ? c0 + u : NL - 1;
            if (c0 + u >= k && c0 + u < NL) q1[c] = fma(-tau * dot[u], vk, q1[c]);
          }
        }
      };
      StaticFor<0, (NL + CH - 1) / CH>::run(chunk);
    };
    StaticFor<0, NL>::run(orth);
    wave_sync();
    // column r of the pseudo-inverse: D^-1 R^-1 (row r of Q1)^T
    if (valid && row[0] < NE1) {
      auto back = [&](auto kc) {
        constexpr int k = NL - 1 - decltype(kc)::value;
        double s = q1[k];
#pragma unroll
        for (int c = k + 1; c < NL; ++c) s = fma(-L[OR + k * NL + c], q1[c], s);
        q1[k] = s / L[ORD + k];
      };
      StaticFor<0, NL>::run(back);
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const double x = q1[l] / L[OSC + l];
        const int64_t at = ((int64_t)row[0] * NL + l) * p.Np + i;
        if (p.pinv64) p.pinv64[at] = x;
        if (p.pinv32) p.pinv32[at] = (float)x;
      }
    }
    if (valid && sl < NS) {
#pragma unroll
      for (int l = 0; l < D; ++l)
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const int64_t at = (int64_t)((sl * D + l) * D + a) * p.Np + i;
          const double x = L[OBI + (sl * D + l) * D + a];
          if (p.binv64) p.binv64[at] = x;
          if (p.binv32) p.binv32[at] = (float)x;
        }
    }
    if (valid && sl == 0 && p.mask) p.mask[i] = (uint8_t)kmask;
    (void)inv_l0;
  } else {
  // 5. variable blocks
  for (int v0 = 0; v0 < p.nv; v0 += VB) {
    const int nvb = min(VB, p.nv - v0);
    double dq[RPL][VB];
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      const bool act = v < nvb;
      const T* qv = p.q + (int64_t)(act ? v0 + v : v0) * nc;
      const double qi = (double)qv[ic];
#pragma unroll
      for (int t = 0; t < RPL; ++t) dq[t][v] = (act && rv[t]) ? (double)qv[jr[t]] - qi : 0.0;
    }
    // the blend lane's own average and its sector cells' averages: gathered
    // before the reflections where the kernel runs one wave per SIMD (the
    // 3-D degree >= 3 shapes, whose latency no other wave hides), else at
    // the blend (the registers they would hold meanwhile cost a wave)
    constexpr bool kEarly = D == 3 && M >= 3;
    T qiT = T(0);
    double qsec[NS][D];
    auto gather_blend = [&](int v) {
      const T* qv = p.q + (int64_t)v * nc;
      qiT = qv[ic];
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int a = 0; a < D; ++a) qsec[s][a] = (double)qv[LJ[s * D + a]];
    };
    if constexpr (kEarly) gather_blend(v0 + (sl < nvb ? sl : 0));
    auto reflect = [&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const double tau = L[OTAU + k];
      double vk[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) vk[t] = row[t] >= k ? A[t][k] : 0.0;
      double dd[VB];
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) s = fma(vk[t], dq[t][v], s);
        dd[v] = s;
      }
      seg_sum<SEG, VB>(dd, 0);
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        const double f = -tau * dd[v];
#pragma unroll
        for (int t = 0; t < RPL; ++t) dq[t][v] = fma(f, vk[t], dq[t][v]);
      }
    };
    StaticFor<0, NL>::run(reflect);
    // back substitution R x = Q^T dQ over the row lanes: x_k is formed from
    // the lane of row k, broadcast, and removed from the rows above it
    auto back = [&](auto kc) {
      constexpr int k = NL - 1 - decltype(kc)::value;
      const double ik = rcp_nz(L[ORD + k]);
      double xk[VB];
#pragma unroll
      for (int v = 0; v < VB; ++v) xk[v] = seg_bcast<SEG, k % SEG>(dq[k / SEG][v], seg) * ik;
#pragma unroll
      for (int t = 0; t <= k / SEG; ++t)
        if (row[t] < k) {
          const double rk = A[t][k];
#pragma unroll
          for (int v = 0; v < VB; ++v) dq[t][v] = fma(-rk, xk[v], dq[t][v]);
        }
    };
    StaticFor<0, NL>::run(back);
    // P_opt coefficient r of each variable (column scale undone), to LDS
#pragma unroll
    for (int t = 0; t < RPL; ++t)
      if (t * SEG < NL && row[t] < NL) {
        const double f = rcp_nz(L[ORD + row[t]] * L[OSC + row[t]]);
#pragma unroll
        for (int v = 0; v < VB; ++v) L[OP + v * NL + row[t]] = dq[t][v] * f;
      }
    wave_sync();
    if (valid && sl < nvb) {
      const int v = v0 + sl;
      if constexpr (!kEarly) gather_blend(v);
      const double qi = (double)qiT;
      double po[NL];
#pragma unroll
      for (int l = 0; l < NL; ++l) po[l] = L[OP + sl * NL + l];
      // sectorial P1 polynomials
      double ps[NS][D];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        double dqs[D];
#pragma unroll
        for (int a = 0; a < D; ++a) dqs[a] = qsec[s][a] - qi;
#pragma unroll
        for (int l = 0; l < D; ++l) {
          double x = 0.0;
#pragma unroll
          for (int a = 0; a < D; ++a) x = fma(L[OBI + (s * D + l) * D + a], dqs[a], x);
          ps[s][l] = x;
        }
      }
      // P_0 = (P_opt - sum_s lambda_s P_s) / lambda_0, kept as u = lambda_0 P_0
      const bool s_popt = p.sigma0_popt;
      double u[D];
#pragma unroll
      for (int l = 0; l < D; ++l) {
        double x = po[l];
#pragma unroll
        for (int s = 0; s < NS; ++s) x = fma(-lam[s + 1], ps[s][l], x);
        u[l] = x;
        po[l] = s_popt ? po[l] : x;
      }
      double sg[NS + 1];
      sg[0] = quad_form<D, M, double>(po) * (s_popt ? 1.0 : inv_l0 * inv_l0);
#pragma unroll
      for (int l = 0; l < D; ++l) po[l] = u[l];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        double x = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) {
          double y = 0.0;
#pragma unroll
          for (int m = l + 1; m < D; ++m) y = fma(SigmaTable<D, M>::v[l * NL + m], ps[s][m], y);
          x = fma(ps[s][l], fma(2.0, y, SigmaTable<D, M>::v[l * NL + l] * ps[s][l]), x);
        }
        sg[s + 1] = x;
      }
      double om[NS + 1];
      if (p.linear_w) {
#pragma unroll
        for (int s = 0; s <= NS; ++s) om[s] = lam[s];
      } else {
        double ms[NS + 1];
#pragma unroll
        for (int s = 0; s <= NS; ++s) ms[s] = sg[s] + p.eps;
        double mmin = ms[0];
#pragma unroll
        for (int s = 1; s <= NS; ++s)
          if (lam[s] > 0.0) mmin = fmin(mmin, ms[s]);
#pragma unroll
        // every kept ratio is at most 1, so its power cannot overflow; a
        // dropped sector (lambda_s = 0, sigma_s = 0) gets ratio 0, since
        // (m_min / eps)^r overflows for large r or data, and inf * 0 is NaN
        for (int s = 0; s <= NS; ++s) om[s] = lam[s] > 0.0 ? mmin * rcp_pos(ms[s]) : 0.0;
        powi<NS + 1, double>(om, p.r);
        double tot = 0.0;
#pragma unroll
        for (int s = 0; s <= NS; ++s) {
          om[s] *= lam[s];
          tot += om[s];
        }
        const double itot = rcp_pos(tot);
#pragma unroll
        for (int s = 0; s <= NS; ++s) om[s] *= itot;
      }
      T* o = p.out + (int64_t)v * NB * nc + i;
      o[0] = qiT;
      const double c0 = om[0] * inv_l0;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        double x = c0 * po[l];
        if (l < D) {
#pragma unroll
          for (int s = 0; s < NS; ++s) x = fma(om[s + 1], ps[s][l < D ? l : 0], x);
        }
        o[(int64_t)(l + 1) * nc] = (T)x;
      }
      if (p.sig) {
        T* g = p.sig + (int64_t)v * (NS + 1) * nc + i;
#pragma unroll
        for (int s = 0; s <= NS; ++s) g[(int64_t)s * nc] = (T)sg[s];
      }
      if (p.om) {
        T* g = p.om + (int64_t)v * (NS + 1) * nc + i;
#pragma unroll
        for (int s = 0; s <= NS; ++s) g[(int64_t)s * nc] = (T)om[s];
      }
    }
    wave_sync();
  }
  }
  if (fault && valid && p.fault) atomicOr(p.fault, fault);
}

}  // namespace cweno
