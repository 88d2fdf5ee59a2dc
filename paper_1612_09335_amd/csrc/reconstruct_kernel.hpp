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
// so the lanes of a wavefront read contiguous runs.  Every load
// is a wave-uniform base (scalar registers) plus a 32-bit per-lane byte
// offset; the host guarantees that the offsets fit (rows of at most 4 GiB).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cweno {

constexpr int kThreads = 256;

__host__ __device__ constexpr int nbasis_c(int M, int D) {
  return D == 2 ? (M + 1) * (M + 2) / 2 : (M + 1) * (M + 2) * (M + 3) / 6;
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
};

// Every array also reaches a kernel as an argument of its own, marked
// __restrict__: the arrays never overlap (the library rejects overlapping
// caller buffers), and saying so lets the compiler keep the sector operators
// in registers and read the universal Sigma through the scalar cache instead
// of reloading both after every store of a coefficient.  A kernel rebinds the
// fields of its KParams to these arguments on entry.
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

// Blocks are dispatched round-robin over the 8 XCDs; renumber them so that
// each XCD sweeps one contiguous range of cells and the neighbour gathers of
// consecutive blocks hit the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

template <typename T>
__device__ __forceinline__ T powi(T x, int r) {
  T y = x;
  for (int t = 1; t < r; ++t) y *= x;
  return y;
}

__host__ __device__ constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Load from a wave-uniform base plus a 32-bit per-lane byte offset.
template <typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Sector differences Q_j - Q_i of variable v gathered from global memory.
template <int D, typename T>
__device__ __forceinline__ void sector_dq_global(const KParams<T>& p, int v, T qi, const int32_t (&sj)[D + 1][D],
                                                 T (&dqs)[D + 1][D]) {
  const T* __restrict__ q = p.q + (int64_t)(p.v0 + v) * p.nc;
#pragma unroll
  for (int s = 0; s <= D; ++s)
#pragma unroll
    for (int a = 0; a < D; ++a) dqs[s][a] = ldo(q, (uint32_t)sj[s][a] * (uint32_t)sizeof(T)) - qi;
}

// Steps (b)-(e) for one cell and one variable, given P_opt's coefficients
// 1..NB-1 as popt(l) and the sector differences dqs[s][a] = Q_{j^s(a)} - Q_i.
template <int D, int M, typename T, class PoptFn>
__device__ __forceinline__ void finish_variable(const KParams<T>& p, int64_t i, int v, T qi, PoptFn popt,
                                                const T (&lam)[D + 2], T inv_l0, const T (&dqs)[D + 1][D]) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NS = D + 1;
  const int64_t qs = p.nc, Np = p.Np;
  const uint32_t io = (uint32_t)i * (uint32_t)sizeof(T);
  // (b) sectorial P1 polynomials
  T ps[NS][D];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int l = 0; l < D; ++l) {
      T x = T(0);
#pragma unroll
      for (int a = 0; a < D; ++a) x = fma(ldo(p.binv + ((s * D + l) * D + a) * Np, io), dqs[s][a], x);
      ps[s][l] = x;
    }
  }
  // (c) P_0
  T p0[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    T x = popt(l);
    if (l < D) {
#pragma unroll
      for (int s = 0; s < NS; ++s) x = fma(-lam[s + 1], ps[s][l], x);
    }
    p0[l] = x * inv_l0;
  }
  // (d) oscillation indicators (Sigma is symmetric)
  const T* __restrict__ Sg = p.sigma;
  T sg[NS + 1];
  {
    T x = T(0);
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const T pl = p.sigma0_popt ? popt(l) : p0[l];
      T y = T(0);
#pragma unroll
      for (int m = l + 1; m < NL; ++m) y = fma(Sg[l * NL + m], p.sigma0_popt ? popt(m) : p0[m], y);
      x = fma(pl, fma(T(2), y, Sg[l * NL + l] * pl), x);
    }
    sg[0] = x;
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    T x = T(0);
#pragma unroll
    for (int l = 0; l < D; ++l) {
      T y = T(0);
#pragma unroll
      for (int m = l + 1; m < D; ++m) y = fma(Sg[l * NL + m], ps[s][m], y);
      x = fma(ps[s][l], fma(T(2), y, Sg[l * NL + l] * ps[s][l]), x);
    }
    sg[s + 1] = x;
  }
  // (e) nonlinear weights and blend
  T om[NS + 1];
  if (p.linear_w) {
#pragma unroll
    for (int s = 0; s <= NS; ++s) om[s] = lam[s];
  } else {
    T dmin = sg[0] + p.eps;
#pragma unroll
    for (int s = 1; s <= NS; ++s)
      if (lam[s] > T(0)) dmin = fmin(dmin, sg[s] + p.eps);
    T tot = T(0);
#pragma unroll
    for (int s = 0; s <= NS; ++s) {
      om[s] = lam[s] * powi(dmin / (sg[s] + p.eps), p.r);
      tot += om[s];
    }
    const T inv = T(1) / tot;
#pragma unroll
    for (int s = 0; s <= NS; ++s) om[s] *= inv;
  }
  T* o = p.out + (int64_t)(p.v0 + v) * NB * qs + i;
  o[0] = qi;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    T x = om[0] * p0[l];
    if (l < D) {
#pragma unroll
      for (int s = 0; s < NS; ++s) x = fma(om[s + 1], ps[s][l], x);
    }
    o[(int64_t)(l + 1) * qs] = x;
  }
  if (p.sig) {
    T* so = p.sig + ((int64_t)(p.v0 + v) * (NS + 1)) * qs + i;
#pragma unroll
    for (int s = 0; s <= NS; ++s) so[(int64_t)s * qs] = sg[s];
  }
  if (p.om) {
    T* oo = p.om + ((int64_t)(p.v0 + v) * (NS + 1)) * qs + i;
#pragma unroll
    for (int s = 0; s <= NS; ++s) oo[(int64_t)s * qs] = om[s];
  }
}

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

  const uint32_t io = (uint32_t)i * (uint32_t)sizeof(T);
  const uint32_t io4 = (uint32_t)i * 4u;
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
    gc[kk] = kk < NE1 ? (uint32_t)ldo(p.gidx + (int64_t)kk * Np, io4) : (uint32_t)i;
  for (int k0 = 0; k0 < NE1; k0 += KC) {
    uint32_t gn[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = k0 + KC + kk;
      gn[kk] = k < NE1 ? (uint32_t)ldo(p.gidx + (int64_t)k * Np, io4) : (uint32_t)i;
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
      const T* __restrict__ row = p.pinv + (int64_t)k * NL * Np;
#pragma unroll
      for (int l = 0; l < NL; ++l) rr[kk][l] = k < NE1 ? ldo(row + (int64_t)l * Np, io) : T(0);
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

  // Linear weights of this cell: dropped sectors get 0, the rest renormalised.
  const unsigned mask = ldo(p.mask, (uint32_t)i);
  T lam[NS + 1];
  T lsum = p.lam[0];
  lam[0] = p.lam[0];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    lam[s + 1] = ((mask >> s) & 1u) ? p.lam[s + 1] : T(0);
    lsum += lam[s + 1];
  }
#pragma unroll
  for (int s = 0; s <= NS; ++s) lam[s] /= lsum;
  const T inv_l0 = T(1) / lam[0];
  int32_t sj[NS][D];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const uint32_t pos = ldo(p.secpos + (s * D + a) * Np, (uint32_t)i);
      sj[s][a] = ldo(p.gidx + (int64_t)pos * Np, io4);
    }
#pragma unroll
  for (int v = 0; v < VB; ++v) {
    T dqs[NS][D];
    sector_dq_global<D, T>(p, v, qi[v], sj, dqs);
    finish_variable<D, M, T>(p, i, v, qi[v], [&](int l) { return acc[l][v]; }, lam, inv_l0, dqs);
  }
}

}  // namespace cweno
