// CWENO reconstruction kernel for gfx950 (CDNA4).
//
// Per cell i and variable v (Sec. 2.1):
//   (a) P_opt: p_0 = Q_i, p_{1..} = pinv_i (Q_{j(k)} - Q_i)        eq. CWENO:Popt
//   (b) sector s: p_0 = Q_i, p_{1..d} = binv_{i,s} (Q_{j^s(a)} - Q_i) eq. CWENO:Ps
//   (c) P_0 = (P_opt - sum_s lambda_s P_s) / lambda_0                eq. CWENO:P0
//   (d) sigma_s = p_s^T Sigma p_s (the constant coefficient does not enter)
//   (e) omega~_s = lambda_s / (sigma_s + eps)^r, normalised; w = sum_s omega_s P_s
//       (eqs. weights, weights2, CWENO:Prec).  The weights are formed as
//       lambda_s * ((sigma_min + eps) / (sigma_s + eps))^r, the same numbers
//       after normalisation, but free of overflow and of the underflow of
//       (sigma + eps)^r in single precision.
// Coefficient 0 of the result is a bitwise copy of Q_i (conservation).
//
// Work mapping.  One lane per cell; the lane keeps (NB-1) * VB accumulators
// for the VB variables of the block, so each operator entry is read from HBM
// exactly once.  The stencil is walked in chunks of KC entries: the gather
// indices of the next chunk are loaded while the current chunk's neighbour
// averages and operator rows are in flight.
//
// Memory layout (structure of arrays, cell index fastest, row stride Np):
//   pinv[(k * (NB-1) + l) * Np + i]   k < NE1, l < NB-1
//   binv[((s * D + l) * D + a) * Np + i]
//   gidx[k * Np + i] (int32)        k < G: stencil cells then sector extras
//   secpos[(s * D + a) * Np + i] (uint8), mask[i] (uint8, bit s = sector alive)
//   q[v * qs + i], out[(v * NB + l) * qs + i] with qs = n_cells
// so the lanes of a wavefront read contiguous runs.
//
// Addressing.  The operator rows, index rows and coefficient rows are read and
// written through buffer resources: a wave-uniform 64-bit base in scalar
// registers, a wave-uniform row offset in a scalar register and the lane's
// 32-bit byte offset, so that no vector instruction is spent on addresses.
// The host guarantees that every such offset fits in 32 bits.  The universal
// Sigma of (D, M) is a table of compile-time constants (generated at build
// time), folded into the instructions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sigma_tables.hpp"   // generated at build time by gen_sigma.cpp

namespace cweno {

constexpr int kThreads = 256;
constexpr int kHaloBlockLanes = 256;   // threads of a halo-kernel workgroup (one cell each)

__host__ __device__ constexpr int nbasis_c(int M, int D) {
  return D == 2 ? (M + 1) * (M + 2) / 2 : (M + 1) * (M + 2) * (M + 3) / 6;
}

// P_opt accumulators one lane may hold in registers: (NB-1) * VB of them,
// at most 100 doubles or 200 floats.
__host__ __device__ constexpr int acc_budget(bool f32) { return f32 ? 200 : 100; }

// Passes of the LDS-halo kernel over the stencil for one block of VB
// variables: 1 when all (NB-1) * VB accumulators fit the budget, else 2, each
// accumulating half of P_opt's rows (the operator rows are still read once).
__host__ __device__ constexpr int halo_chunks(int D, int M, int VB, bool f32) {
  return (nbasis_c(M, D) - 1) * VB <= acc_budget(f32) ? 1 : 2;
}

template <typename T>
struct KParams {
  const T* q;
  T* out;
  T* sig;          // optional
  T* om;           // optional
  const T* pinv;
  const T* binv;
  const T* sigma;  // (NB-1)^2, uniform across the grid
  const int32_t* gidx;
  const uint8_t* secpos;
  const uint8_t* mask;
  const int32_t* halo;     // concatenated per-block halos (halo kernel)
  const int32_t* hoff;     // [n_blocks + 1]
  const uint16_t* lidx;    // [G+1][Np] gather entries as positions in the block halo; row G: the cell
  int maxH;                // largest halo
  int G;                   // gather-list length
  int64_t nc;      // cells
  int64_t Np;      // operator row stride
  int NE1;         // stencil cells besides i
  int v0;          // first variable of this block
  int r;           // weight exponent
  int sigma0_popt; // indicator of the central polynomial from P_opt
  int linear_w;    // omega := lambda
  T lam[5];        // lambda_0 .. lambda_{d+1}
  T eps;
  // fused point values (the PTS kernels): basis values [npts][NB] and
  // values [nv][npts][nc] written instead of the coefficients
  const T* phi;
  T* pv;
  int npts;
};

// Every array also reaches a kernel as an argument of its own, marked
// __restrict__: the arrays never overlap (the library rejects overlapping
// caller buffers), and saying so lets the compiler keep the sector operators
// in registers instead of reloading them after every store of a coefficient.
// A kernel rebinds the fields of its KParams to these arguments on entry.
#define CWENO_ARRAY_PARAMS(T)                                                                          \
  const T* __restrict__ a_q, T* __restrict__ a_out, T* __restrict__ a_sig, T* __restrict__ a_om,       \
      const T* __restrict__ a_pinv, const T* __restrict__ a_binv, const T* __restrict__ a_sigma,       \
      const int32_t* __restrict__ a_gidx, const uint8_t* __restrict__ a_secpos,                         \
      const uint8_t* __restrict__ a_mask, const int32_t* __restrict__ a_halo,                           \
      const int32_t* __restrict__ a_hoff, const uint16_t* __restrict__ a_lidx
#define CWENO_BIND_ARRAYS(p)                                                                           \
  do {                                                                                                 \
    p.q = a_q; p.out = a_out; p.sig = a_sig; p.om = a_om; p.pinv = a_pinv; p.binv = a_binv;            \
    p.sigma = a_sigma; p.gidx = a_gidx; p.secpos = a_secpos; p.mask = a_mask; p.halo = a_halo;         \
    p.hoff = a_hoff; p.lidx = a_lidx;                                                                  \
  } while (0)
#define CWENO_ARRAY_ARGS(p) \
  p.q, p.out, p.sig, p.om, p.pinv, p.binv, p.sigma, p.gidx, p.secpos, p.mask, p.halo, p.hoff, p.lidx

// ---------------------------------------------------------------- addressing

using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Raw buffer resource over `bytes` bytes from `base` (gfx9 word 3: 32-bit
// untyped data, no swizzle).
__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Cache policy of streams touched once per launch (operator and halo-position
// rows read, coefficient rows written): non-temporal, so that they do not
// evict the neighbour averages that the halo staging re-reads from L2.
constexpr int kStream = 2;

// Load/store at byte offset voff (per lane) + soff (wave-uniform).
template <typename T> __device__ __forceinline__ T bld(rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ double bld<double>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ float bld<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ int32_t bld<int32_t>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}
template <> __device__ __forceinline__ uint16_t bld<uint16_t>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
}
template <> __device__ __forceinline__ uint8_t bld<uint8_t>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, voff, soff, 0);
}
// Operator-row load, streamed (read once per launch).
template <typename T> __device__ __forceinline__ T bld_stream(rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ double bld_stream<double>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kStream));
}
template <> __device__ __forceinline__ float bld_stream<float>(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kStream));
}
// Store that keeps the line in the caches (a value the same lane reads back).
__device__ __forceinline__ void bst_keep(rsrc_t r, double x, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, soff, 0);
}
__device__ __forceinline__ void bst_keep(rsrc_t r, float x, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, voff, soff, 0);
}
// Coefficient-row store, streamed (written once per launch).
__device__ __forceinline__ void bst(rsrc_t r, double x, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, soff, kStream);
}
__device__ __forceinline__ void bst(rsrc_t r, float x, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, voff, soff, kStream);
}

// Load from a wave-uniform base plus a 32-bit per-lane byte offset (gathers).
template <typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// ---------------------------------------------------------------- helpers

// Blocks are dispatched round-robin over the 8 XCDs; renumber them so that
// each XCD sweeps one contiguous range of cells and the neighbour gathers of
// consecutive blocks hit the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

// x[s]^r for the wave-uniform exponent r >= 1; r = 4 (the usual choice)
// without a loop.
template <int N, typename T>
__device__ __forceinline__ void powi(T (&x)[N], int r) {
  if (r == 4) {
#pragma unroll
    for (int s = 0; s < N; ++s) {
      const T x2 = x[s] * x[s];
      x[s] = x2 * x2;
    }
    return;
  }
  T y[N];
#pragma unroll
  for (int s = 0; s < N; ++s) y[s] = x[s];
  for (int t = 1; t < r; ++t)
#pragma unroll
    for (int s = 0; s < N; ++s) y[s] *= x[s];
#pragma unroll
  for (int s = 0; s < N; ++s) x[s] = y[s];
}

__host__ __device__ constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// 1/x for finite x > 0 whose reciprocal is a normal number: the hardware
// estimate refined by Newton steps e = 1 - x r, r += r e (one step in single
// precision, two in double), within an ulp or two of the rounded quotient.
__device__ __forceinline__ float rcp_pos(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double rcp_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// p^T Sigma p over coefficients 1..NL with the universal Sigma of (D, M) as
// compile-time constants (symmetric: each off-diagonal product once, doubled).
template <int D, int M, typename T>
__device__ __forceinline__ T quad_form(const T (&pv)[nbasis_c(M, D) - 1]) {
  constexpr int NL = nbasis_c(M, D) - 1;
  using S = SigmaTable<D, M>;
  T x = T(0);
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    T y = T(0);
#pragma unroll
    for (int m = l + 1; m < NL; ++m) y = fma(T(S::v[l * NL + m]), pv[m], y);
    x = fma(pv[l], fma(T(2), y, T(S::v[l * NL + l]) * pv[l]), x);
  }
  return x;
}

// Per-cell linear weights: dropped sectors (mask bit clear) get 0, the rest
// are renormalised; returns 1 / lambda_0.
template <int NS, typename T>
__device__ __forceinline__ T cell_weights(const KParams<T>& p, unsigned mask, T (&lam)[NS + 1]) {
  T lsum = p.lam[0];
  lam[0] = p.lam[0];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    lam[s + 1] = ((mask >> s) & 1u) ? p.lam[s + 1] : T(0);
    lsum += lam[s + 1];
  }
#pragma unroll
  for (int s = 0; s <= NS; ++s) lam[s] /= lsum;
  return T(1) / lam[0];
}

// The cell's sector operators binv[s][l][a] (loaded once for all variables,
// before the first coefficient store).
template <int D, typename T>
__device__ __forceinline__ void load_binv(const T* binv, int64_t Np, uint32_t io, T (&bv)[D + 1][D][D]) {
  const uint32_t prow = (uint32_t)Np * (uint32_t)sizeof(T);
  const rsrc_t rb = make_rsrc(binv, (uint32_t)((D + 1) * D * D) * prow);
#pragma unroll
  for (int s = 0; s <= D; ++s)
#pragma unroll
    for (int l = 0; l < D; ++l)
#pragma unroll
      for (int a = 0; a < D; ++a) bv[s][l][a] = bld_stream<T>(rb, io, (uint32_t)((s * D + l) * D + a) * prow);
}

// Steps (b)-(e) for one cell and one variable, given P_opt's coefficients
// 1..NB-1 in po (overwritten) and the sector differences
// dqs[s][a] = Q_{j^s(a)} - Q_i.  lam holds the cell's linear weights
// (normalised), inv_l0 = 1 / lam[0].  io is the lane's byte offset of its
// cell in an operator or coefficient row.
template <int D, int M, typename T, bool PTS = false>
__device__ __forceinline__ void finish_variable(const KParams<T>& p, uint32_t io, int v, T qi,
                                                T (&po)[nbasis_c(M, D) - 1], const T (&lam)[D + 2], T inv_l0,
                                                const T (&dqs)[D + 1][D], const T (&bv)[D + 1][D][D],
                                                T* lw = nullptr) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NS = D + 1;
  const int64_t qs = p.nc, Np = p.Np;
  const uint32_t prow = (uint32_t)Np * (uint32_t)sizeof(T);   // operator row, bytes
  const uint32_t crow = (uint32_t)qs * (uint32_t)sizeof(T);   // coefficient row, bytes
  // (b) sectorial P1 polynomials
  T ps[NS][D];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int l = 0; l < D; ++l) {
      T x = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) x = fma(bv[s][l][a], dqs[s][a], x);
      ps[s][l] = x;
    }
  // (c) P_0 = u / lambda_0 with u = P_opt - sum_s lambda_s P_s; only the
  // linear coefficients differ from P_opt's.  (d) oscillation indicators,
  // sigma(P_0) = sigma(u) / lambda_0^2 (or sigma(P_opt) on request).
  const bool s_popt = p.sigma0_popt;
  T u[D];
#pragma unroll
  for (int l = 0; l < D; ++l) {
    T x = po[l];
#pragma unroll
    for (int s = 0; s < NS; ++s) x = fma(-lam[s + 1], ps[s][l], x);
    u[l] = x;
    po[l] = s_popt ? po[l] : x;
  }
  T sg[NS + 1];
  sg[0] = quad_form<D, M, T>(po) * (s_popt ? T(1) : inv_l0 * inv_l0);
#pragma unroll
  for (int l = 0; l < D; ++l) po[l] = u[l];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    T x = T(0);
#pragma unroll
    for (int l = 0; l < D; ++l) {
      T y = T(0);
#pragma unroll
      for (int m = l + 1; m < D; ++m) y = fma(T(SigmaTable<D, M>::v[l * NL + m]), ps[s][m], y);
      x = fma(ps[s][l], fma(T(2), y, T(SigmaTable<D, M>::v[l * NL + l]) * ps[s][l]), x);
    }
    sg[s + 1] = x;
  }
  // (e) nonlinear weights lambda_s (m_min / m_s)^r normalised, m_s = sigma_s + eps
  T om[NS + 1];
  if (p.linear_w) {
#pragma unroll
    for (int s = 0; s <= NS; ++s) om[s] = lam[s];
  } else {
    T ms[NS + 1];
#pragma unroll
    for (int s = 0; s <= NS; ++s) ms[s] = sg[s] + p.eps;
    T mmin = ms[0];
#pragma unroll
    for (int s = 1; s <= NS; ++s)
      if (lam[s] > T(0)) mmin = fmin(mmin, ms[s]);
    // a dropped sector (lambda_s = 0) gets ratio 0: its sigma is 0, and
    // m_min / eps raised to the power r would overflow in single precision
#pragma unroll
    for (int s = 0; s <= NS; ++s) om[s] = lam[s] > T(0) ? mmin * rcp_pos(ms[s]) : T(0);
    powi<NS + 1, T>(om, p.r);
    T tot = T(0);
#pragma unroll
    for (int s = 0; s <= NS; ++s) {
      om[s] *= lam[s];
      tot += om[s];
    }
    const T inv = rcp_pos(tot);
#pragma unroll
    for (int s = 0; s <= NS; ++s) om[s] *= inv;
  }
  // blend: w = omega_0 P_0 + sum_s omega_s P_s; coefficient 0 is Q_i itself
  const T c0 = om[0] * inv_l0;
  if constexpr (!PTS) {
    const rsrc_t ro = make_rsrc(p.out + (int64_t)(p.v0 + v) * NB * qs, NB * crow);
    bst(ro, qi, io, 0u);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      T x = c0 * po[l];
      if (l < D) {
#pragma unroll
        for (int s = 0; s < NS; ++s) x = fma(om[s + 1], ps[s][l < D ? l : 0], x);
      }
      bst(ro, x, io, (uint32_t)(l + 1) * crow);
    }
  } else {
    // the polynomial's values at the point set instead of its coefficients,
    // summed in the order of the evaluation kernel (same bits); the blended
    // coefficients wait in the lane's LDS column lw[l * kHaloBlock] so that
    // they hold no registers while the other variables' sums are live, and
    // the basis values at the points, the same for every lane, are read
    // through the constant address space (scalar loads into SGPRs)
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      T x = c0 * po[l];
      if (l < D) {
#pragma unroll
        for (int s = 0; s < NS; ++s) x = fma(om[s + 1], ps[s][l < D ? l : 0], x);
      }
      lw[l * kHaloBlockLanes] = x;
    }
    const rsrc_t rp = make_rsrc(p.pv + (int64_t)(p.v0 + v) * p.npts * qs, (uint32_t)p.npts * crow);
    T w[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) w[l] = lw[l * kHaloBlockLanes];
    using cT = __attribute__((address_space(4))) const T;
    const cT* const phi = (const cT*)p.phi;
    // two points per step: the second point's basis values are requested
    // with the first's, so one scalar-load round trip serves both
    int q = 0;
    for (; q + 1 < p.npts; q += 2) {
      const cT* f = phi + q * NB;
      const cT* g = f + NB;
      T x = fma(f[0], qi, T(0)), y = fma(g[0], qi, T(0));
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        x = fma(f[l + 1], w[l], x);
        y = fma(g[l + 1], w[l], y);
      }
      bst(rp, x, io, (uint32_t)q * crow);
      bst(rp, y, io, (uint32_t)(q + 1) * crow);
    }
    if (q < p.npts) {
      const cT* f = phi + q * NB;
      T x = fma(f[0], qi, T(0));
#pragma unroll
      for (int l = 0; l < NL; ++l) x = fma(f[l + 1], w[l], x);
      bst(rp, x, io, (uint32_t)q * crow);
    }
  }
  if (p.sig) {
    const rsrc_t rs = make_rsrc(p.sig + (int64_t)(p.v0 + v) * (NS + 1) * qs, (NS + 1) * crow);
#pragma unroll
    for (int s = 0; s <= NS; ++s) bst(rs, sg[s], io, (uint32_t)s * crow);
  }
  if (p.om) {
    const rsrc_t rw = make_rsrc(p.om + (int64_t)(p.v0 + v) * (NS + 1) * qs, (NS + 1) * crow);
#pragma unroll
    for (int s = 0; s <= NS; ++s) bst(rw, om[s], io, (uint32_t)s * crow);
  }
}

// ---------------------------------------------------------------- direct kernel

template <int D, int M, int VB, int KC, typename T>
__global__ __launch_bounds__(kThreads) void reconstruct_kernel(KParams<T> p, CWENO_ARRAY_PARAMS(T)) {
  CWENO_BIND_ARRAYS(p);
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NS = D + 1;
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (i >= p.nc) return;
  const int64_t Np = p.Np, qs = p.nc;
  const T* __restrict__ q = p.q + (int64_t)p.v0 * qs;
  const uint32_t prow = (uint32_t)Np * (uint32_t)sizeof(T);
  const uint32_t irow = (uint32_t)Np * 4u;

  const uint32_t io = (uint32_t)i * (uint32_t)sizeof(T);
  const uint32_t io4 = (uint32_t)i * 4u;
  const rsrc_t rg = make_rsrc(p.gidx, (uint32_t)p.G * irow);
  T qi[VB];
#pragma unroll
  for (int v = 0; v < VB; ++v) qi[v] = ldo(q + v * qs, io);

  T acc[NL][VB];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int v = 0; v < VB; ++v) acc[l][v] = T(0);

  // (a) P_opt, stencil walked in chunks of KC
  const int NE1 = p.NE1;
  uint32_t gc[KC];
#pragma unroll
  for (int kk = 0; kk < KC; ++kk)
    gc[kk] = kk < NE1 ? (uint32_t)bld<int32_t>(rg, io4, (uint32_t)kk * irow) : (uint32_t)i;
  for (int k0 = 0; k0 < NE1; k0 += KC) {
    uint32_t gn[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = k0 + KC + kk;
      gn[kk] = k < NE1 ? (uint32_t)bld<int32_t>(rg, io4, (uint32_t)k * irow) : (uint32_t)i;
    }
    T dq[KC][VB];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int v = 0; v < VB; ++v) dq[kk][v] = ldo(q + v * qs, gc[kk] * (uint32_t)sizeof(T)) - qi[v];
    T rr[KC][NL];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = k0 + kk;
      const rsrc_t rk = make_rsrc(p.pinv + (int64_t)k * NL * Np, NL * prow);
#pragma unroll
      for (int l = 0; l < NL; ++l) rr[kk][l] = k < NE1 ? bld_stream<T>(rk, io, (uint32_t)l * prow) : T(0);
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int v = 0; v < VB; ++v) acc[l][v] = fma(rr[kk][l], dq[kk][v], acc[l][v]);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) gc[kk] = gn[kk];
  }

  const rsrc_t rsp = make_rsrc(p.secpos, (uint32_t)(NS * D) * (uint32_t)Np);
  const unsigned mask = ldo(p.mask, (uint32_t)i);
  T lam[NS + 1];
  const T inv_l0 = cell_weights<NS, T>(p, mask, lam);
  int32_t sj[NS][D];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const uint32_t pos = bld<uint8_t>(rsp, (uint32_t)i, (uint32_t)(s * D + a) * (uint32_t)Np);
      sj[s][a] = bld<int32_t>(rg, io4, pos * irow);
    }
  T bv[NS][D][D];
  load_binv<D, T>(p.binv, Np, io, bv);
#pragma unroll
  for (int v = 0; v < VB; ++v) {
    const T* __restrict__ qv = q + v * qs;
    T dqs[NS][D];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int a = 0; a < D; ++a) dqs[s][a] = ldo(qv, (uint32_t)sj[s][a] * (uint32_t)sizeof(T)) - qi[v];
    T po[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) po[l] = acc[l][v];
    finish_variable<D, M, T>(p, io, v, qi[v], po, lam, inv_l0, dqs, bv);
  }
}

}  // namespace cweno
