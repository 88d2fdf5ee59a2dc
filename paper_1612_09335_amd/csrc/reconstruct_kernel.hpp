// CWENO reconstruction kernel for gfx950 (CDNA4).
//
// One thread per cell; a thread handles a block of VB variables so that the
// per-cell operators are streamed from HBM once per block.  Per cell i and
// variable v (Sec. 2.1):
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
// Memory layout (structure of arrays, cell index fastest, row stride Np):
//   pinv[(l * NE1 + k) * Np + i]   l < NB-1, k < NE1
//   binv[((s * D + l) * D + a) * Np + i]
//   gidx[k * Np + i] (int32)        k < G: stencil cells then sector extras
//   secpos[(s * D + a) * Np + i] (uint8), mask[i] (uint8, bit s = sector alive)
//   q[v * qs + i], out[(v * NB + l) * qs + i] with qs = n_cells
// so every operator load of a wavefront reads 64 consecutive cells.
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

template <int D, int M, int VB, typename T>
__global__ __launch_bounds__(kThreads) void reconstruct_kernel(KParams<T> p) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NS = D + 1;
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (i >= p.nc) return;
  const int64_t Np = p.Np, qs = p.nc;
  const T* __restrict__ q = p.q + (int64_t)p.v0 * qs;

  T qi[VB];
#pragma unroll
  for (int v = 0; v < VB; ++v) qi[v] = q[v * qs + i];

  // (a) P_opt: acc = pinv * dQ, streaming the operator column by column.
  T acc[NL][VB];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int v = 0; v < VB; ++v) acc[l][v] = T(0);

  const int32_t* __restrict__ gidx = p.gidx + i;
  const T* __restrict__ pinv = p.pinv + i;
  const int NE1 = p.NE1;
#pragma unroll 1
  for (int k = 0; k < NE1; ++k) {
    const int64_t j = gidx[k * Np];
    T dq[VB];
#pragma unroll
    for (int v = 0; v < VB; ++v) dq[v] = q[v * qs + j] - qi[v];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const T rl = pinv[(int64_t)(l * NE1 + k) * Np];
#pragma unroll
      for (int v = 0; v < VB; ++v) acc[l][v] = fma(rl, dq[v], acc[l][v]);
    }
  }

  // Linear weights of this cell: dropped sectors get 0, the rest renormalised.
  const unsigned mask = p.mask[i];
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

  // Sector cells (indices into the gather list) and their inverse matrices.
  int32_t sj[NS][D];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int a = 0; a < D; ++a) sj[s][a] = gidx[(int64_t)p.secpos[(s * D + a) * Np + i] * Np];

  const T* __restrict__ Sg = p.sigma;
  T* __restrict__ out = p.out + (int64_t)p.v0 * NB * qs;

#pragma unroll
  for (int v = 0; v < VB; ++v) {
    // (b) sectorial P1 polynomials
    T ps[NS][D];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      T dqs[D];
#pragma unroll
      for (int a = 0; a < D; ++a) dqs[a] = q[v * qs + sj[s][a]] - qi[v];
#pragma unroll
      for (int l = 0; l < D; ++l) {
        T x = T(0);
#pragma unroll
        for (int a = 0; a < D; ++a) x = fma(p.binv[((s * D + l) * D + a) * Np + i], dqs[a], x);
        ps[s][l] = x;
      }
    }
    // (c) P_0
    T p0[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      T x = acc[l][v];
      if (l < D) {
#pragma unroll
        for (int s = 0; s < NS; ++s) x = fma(-lam[s + 1], ps[s][l], x);
      }
      p0[l] = x * inv_l0;
    }
    // (d) oscillation indicators
    T sg[NS + 1];
    {
      T x = T(0);
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        T y = T(0);
#pragma unroll
        for (int m = 0; m < NL; ++m) y = fma(Sg[l * NL + m], p.sigma0_popt ? acc[m][v] : p0[m], y);
        x = fma(p.sigma0_popt ? acc[l][v] : p0[l], y, x);
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
        for (int m = 0; m < D; ++m) y = fma(Sg[l * NL + m], ps[s][m], y);
        x = fma(ps[s][l], y, x);
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
    T* o = out + (int64_t)v * NB * qs + i;
    o[0] = qi[v];
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
}

}  // namespace cweno
