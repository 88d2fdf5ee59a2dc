// LDS-halo variant of the CWENO reconstruction kernel (gfx950).
//
// Same arithmetic as reconstruct_kernel (one lane per cell; each P_opt row a
// FMA chain over the stencil in order k = 0, 1, ...; identical epilogue).
//
// Neighbour gathers are what limits the direct kernels: every stencil entry
// of 64 lanes is a scattered load, and the texture-data return path spends
// far longer on it than on a coalesced operator row.  Consecutive cells share
// most of their stencil cells, so a workgroup of 256 consecutive cells first
// copies the averages of its halo -- the sorted unique cells its gather lists
// reference, precomputed on the host -- into LDS (each cell once, mostly in
// contiguous runs), and then reads every stencil and sector value from LDS
// through 16-bit halo positions.  The operator rows keep streaming from HBM
// in coalesced loads; the 16-bit positions also halve the index stream.
//
// LDS layout: halo values [VB][maxH].
#pragma once

#include "reconstruct_kernel.hpp"

namespace cweno {

constexpr int kHaloBlock = 256;   // cells (and threads) per workgroup; fixed by the host's halo lists

template <int D, int M, int VB, int KC, typename T>
__global__ __launch_bounds__(kHaloBlock) void reconstruct_halo_kernel(KParams<T> p, CWENO_ARRAY_PARAMS(T)) {
  CWENO_BIND_ARRAYS(p);
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NS = D + 1;
  extern __shared__ __align__(16) unsigned char halo_raw[];
  T* const lq = reinterpret_cast<T*>(halo_raw);

  const int tid = (int)threadIdx.x;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int64_t i = b * kHaloBlock + tid;
  const bool valid = i < p.nc;
  const int64_t ic = valid ? i : p.nc - 1;
  const int64_t Np = p.Np, qs = p.nc;
  const int maxH = p.maxH;
  const T* __restrict__ q = p.q + (int64_t)p.v0 * qs;
  const uint32_t io = (uint32_t)ic * (uint32_t)sizeof(T);
  const uint32_t io2 = (uint32_t)ic * 2u;
  (void)io;

  // stage the block's halo averages
  const int h0 = p.hoff[b], hn = p.hoff[b + 1] - h0;
  for (int t = tid; t < hn; t += kHaloBlock) {
    const uint32_t j = (uint32_t)p.halo[h0 + t];
#pragma unroll
    for (int v = 0; v < VB; ++v) lq[v * maxH + t] = ldo(q + v * qs, j * (uint32_t)sizeof(T));
  }

  // the cell itself is in its block's halo: its averages are read from LDS when needed
  const uint32_t self = ldo(p.lidx + (int64_t)p.G * Np, io2);
  uint32_t sl[NS][D];     // halo positions of the sector cells
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const uint32_t pos = ldo(p.secpos + (s * D + a) * Np, (uint32_t)ic);
      sl[s][a] = ldo(p.lidx + (int64_t)pos * Np, io2);
    }
  const unsigned mask = ldo(p.mask, (uint32_t)ic);
  __syncthreads();

  T acc[NL][VB];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int v = 0; v < VB; ++v) acc[l][v] = T(0);

  // (a) P_opt, stencil walked in chunks of KC; positions of the next chunk prefetched
  const int NE1 = p.NE1;
  uint32_t hc[KC];
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) hc[kk] = kk < NE1 ? (uint32_t)ldo(p.lidx + (int64_t)kk * Np, io2) : 0u;
  for (int k0 = 0; k0 < NE1; k0 += KC) {
    uint32_t hn_[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = k0 + KC + kk;
      hn_[kk] = k < NE1 ? (uint32_t)ldo(p.lidx + (int64_t)k * Np, io2) : 0u;
    }
    T rr[KC][NL];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int k = k0 + kk;
      const T* __restrict__ row = p.pinv + (int64_t)k * NL * Np;
#pragma unroll
      for (int l = 0; l < NL; ++l)
        rr[kk][l] = k < NE1 ? ldo(row + (int64_t)l * Np, io) : T(0);
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      T dq[VB];
#pragma unroll
      for (int v = 0; v < VB; ++v) dq[v] = lq[v * maxH + hc[kk]] - lq[v * maxH + self];
#pragma unroll
      for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int v = 0; v < VB; ++v) acc[l][v] = fma(rr[kk][l], dq[v], acc[l][v]);
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) hc[kk] = hn_[kk];
  }

  // Linear weights of this cell: dropped sectors get 0, the rest renormalised.
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
  if (!valid) return;
#pragma unroll
  for (int v = 0; v < VB; ++v) {
    const T qi = lq[v * maxH + self];
    T dqs[NS][D];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int a = 0; a < D; ++a) dqs[s][a] = lq[v * maxH + sl[s][a]] - qi;
    finish_variable<D, M, T>(p, i, v, qi, [&](int l) { return acc[l][v]; }, lam, inv_l0, dqs);
  }
}

}  // namespace cweno
