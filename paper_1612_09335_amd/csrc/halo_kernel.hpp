// LDS-halo variant of the CWENO reconstruction kernel (gfx950).
//
// Same arithmetic as reconstruct_kernel (one lane per cell; each P_opt row a
// FMA chain over the stencil in order k = 0, 1, ...; identical epilogue).
//
// Neighbour gathers are what limits the direct kernel: every stencil entry
// of 64 lanes is a scattered load, and the texture-data return path spends
// far longer on it than on a coalesced operator row.  Consecutive cells share
// most of their stencil cells, so a workgroup of 256 consecutive cells first
// copies the averages of its halo -- the sorted unique cells its gather lists
// reference, precomputed on the host -- into LDS (each cell once, mostly in
// contiguous runs), and then reads every stencil and sector value from LDS
// through 16-bit halo positions.  The operator rows keep streaming from HBM
// in coalesced loads; the 16-bit positions also halve the index stream.
//
// The halo is staged HU entries per thread at a time (all index loads, then
// all value loads, then the LDS stores), and the operator rows of the first
// KC stencil entries are requested before the workgroup barrier.
//
// LDS layout: halo values [maxH][VB] (the VB averages of a halo cell
// together, so one address per stencil entry serves every variable).
#pragma once

#include <type_traits>

#include "reconstruct_kernel.hpp"

namespace cweno {

constexpr int kHaloBlock = 256;   // cells (and threads) per workgroup; fixed by the host's halo lists
static_assert(kHaloBlock == kHaloBlockLanes, "one cell per thread of a halo workgroup");

template <int NL, int KC, typename T>
__device__ __forceinline__ void load_rows(T (&r)[KC][NL], const T* pinv, int64_t Np, int NE1, int k0,
                                          uint32_t io) {
  const uint32_t prow = (uint32_t)Np * (uint32_t)sizeof(T);
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    const int k = k0 + kk;
    const rsrc_t rk = make_rsrc(pinv + (int64_t)k * NL * Np, NL * prow);
#pragma unroll
    for (int l = 0; l < NL; ++l) r[kk][l] = k < NE1 ? bld_stream<T>(rk, io, (uint32_t)l * prow) : T(0);
  }
}

// Rows L0 .. L0+NR-1 of the operator rows of stencil entries k0 .. k0+KC-1
// (the rows of P_opt one pass of the stencil walk accumulates).
template <int NL, int NR, int KC, typename T>
__device__ __forceinline__ void load_rows_part(T (&r)[KC][NR], const T* pinv, int64_t Np, int NE1, int k0, int L0,
                                               uint32_t io) {
  const uint32_t prow = (uint32_t)Np * (uint32_t)sizeof(T);
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    const int k = k0 + kk;
    const rsrc_t rk = make_rsrc(pinv + (int64_t)k * NL * Np, NL * prow);
#pragma unroll
    for (int l = 0; l < NR; ++l)
      r[kk][l] = k < NE1 ? bld_stream<T>(rk, io, (uint32_t)(L0 + l) * prow) : T(0);
  }
}

// Halo positions of stencil entries k0 .. k0+KC-1 (a stream read once per
// launch); entries past the stencil point at the cell itself, so that their
// differences are exactly zero.
template <int KC>
__device__ __forceinline__ void load_pos(uint32_t (&h)[KC], rsrc_t rl, uint32_t lrow, int NE1, int k0, uint32_t io2,
                                         uint32_t self) {
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    const int k = k0 + kk;
    h[kk] = k < NE1 ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rl, io2, (uint32_t)k * lrow, kStream) : self;
  }
}

// acc[l][v] += r[kk][l] * (Q_{j(k)} - Q_i) for the KC entries of one chunk
// (entries past the stencil have zero rows and zero differences)
template <int NL, int VB, int KC, typename T>
__device__ __forceinline__ void fma_chunk(T (&acc)[NL][VB], const T (&r)[KC][NL], const uint32_t (&h)[KC],
                                          const T* lq, uint32_t self) {
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    const T* hv = lq + h[kk] * VB;
    const T* sv = lq + self * VB;
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      const T dq = hv[v] - sv[v];
#pragma unroll
      for (int l = 0; l < NL; ++l) acc[l][v] = fma(r[kk][l], dq, acc[l][v]);
    }
  }
}

// One block b of kHaloBlock consecutive cells of the mesh described by p, with
// lq as the block's LDS halo.  Every thread of the workgroup returns normally.
template <int D, int M, int VB, int KC, int HU, typename T, bool PTS = false>
__device__ __forceinline__ void halo_block(const KParams<T>& p, int64_t b, T* lq) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NS = D + 1;
  const int tid = (int)threadIdx.x;
  const int64_t i = b * kHaloBlock + tid;
  const bool valid = i < p.nc;
  const int64_t ic = valid ? i : p.nc - 1;
  const int64_t Np = p.Np, qs = p.nc;
  const int NE1 = p.NE1;
  const uint32_t io = (uint32_t)ic * (uint32_t)sizeof(T);
  const uint32_t io2 = (uint32_t)ic * 2u;
  const uint32_t lrow = (uint32_t)Np * 2u;
  const rsrc_t rl = make_rsrc(p.lidx, (uint32_t)(p.G + 1) * lrow);
  const rsrc_t rq = make_rsrc(p.q + (int64_t)p.v0 * qs, (uint32_t)VB * (uint32_t)qs * (uint32_t)sizeof(T));
  const uint32_t qrow = (uint32_t)qs * (uint32_t)sizeof(T);


  // stage the block's halo averages, HU entries per thread at a time
  const int h0 = p.hoff[b], hn = p.hoff[b + 1] - h0;
  const rsrc_t rh = make_rsrc(p.halo + h0, (uint32_t)hn * 4u);
  for (int t0 = 0; t0 < hn; t0 += HU * kHaloBlock) {
    uint32_t j[HU];
#pragma unroll
    for (int u = 0; u < HU; ++u) {
      const int t = t0 + u * kHaloBlock + tid;
      j[u] = t < hn ? (uint32_t)bld<int32_t>(rh, (uint32_t)t * 4u, 0u) : 0u;
    }
    T val[HU][VB];
#pragma unroll
    for (int u = 0; u < HU; ++u)
#pragma unroll
      for (int v = 0; v < VB; ++v) val[u][v] = bld<T>(rq, j[u] * (uint32_t)sizeof(T), (uint32_t)v * qrow);
#pragma unroll
    for (int u = 0; u < HU; ++u) {
      const int t = t0 + u * kHaloBlock + tid;
      if (t < hn) {
#pragma unroll
        for (int v = 0; v < VB; ++v) lq[t * VB + v] = val[u][v];
      }
    }
  }

  // the cell itself is in its block's halo: its averages are read from LDS when needed
  const uint32_t self = bld<uint16_t>(rl, io2, (uint32_t)p.G * lrow);
  const rsrc_t rsp = make_rsrc(p.secpos, (uint32_t)(NS * D) * (uint32_t)Np);
  uint32_t sl[NS][D];     // halo positions of the sector cells
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const uint32_t pos = bld<uint8_t>(rsp, (uint32_t)ic, (uint32_t)(s * D + a) * (uint32_t)Np);
      sl[s][a] = bld<uint16_t>(rl, io2, pos * lrow);
    }
  const unsigned mask = ldo(p.mask, (uint32_t)ic);

  constexpr int NCH = halo_chunks(D, M, VB, sizeof(T) == 4);
  if constexpr (NCH == 1) {
    // (a) P_opt, stencil walked in chunks of KC entries; the first chunk's rows
    // and positions are requested before the barrier
    T rr[KC][NL];
    uint32_t hc[KC];
    load_rows<NL, KC, T>(rr, p.pinv, Np, NE1, 0, io);
    load_pos<KC>(hc, rl, lrow, NE1, 0, io2, self);
    __syncthreads();

    T acc[NL][VB];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int v = 0; v < VB; ++v) acc[l][v] = T(0);

    fma_chunk<NL, VB, KC, T>(acc, rr, hc, lq, self);
    for (int k0 = KC; k0 < NE1; k0 += KC) {
      load_rows<NL, KC, T>(rr, p.pinv, Np, NE1, k0, io);
      load_pos<KC>(hc, rl, lrow, NE1, k0, io2, self);
      fma_chunk<NL, VB, KC, T>(acc, rr, hc, lq, self);
    }

    T lam[NS + 1];
    const T inv_l0 = cell_weights<NS, T>(p, mask, lam);
    if (valid) {
      T bv[NS][D][D];
      load_binv<D, T>(p.binv, Np, io, bv);
      const T* sv = lq + self * VB;
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        const T qi = sv[v];
        T dqs[NS][D];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int a = 0; a < D; ++a) dqs[s][a] = lq[sl[s][a] * VB + v] - qi;
        T po[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) po[l] = acc[l][v];
        finish_variable<D, M, T, PTS>(p, io, v, qi, po, lam, inv_l0, dqs, bv,
                                      PTS ? lq + (size_t)p.maxH * VB + tid : nullptr);
      }
    }
  } else {
    // (a) P_opt in two walks of the stencil, each accumulating half of its
    // rows for all VB variables (every operator entry is still read once);
    // each half waits in the cell's own coefficient rows 1.. of the output,
    // which the same lane reads back before the epilogue overwrites them
    static_assert(NCH == 2 && !PTS, "two passes over the stencil, coefficients written to the output");
    constexpr int R0 = (NL + 1) / 2;
    const uint32_t crow = (uint32_t)qs * (uint32_t)sizeof(T);
    auto pass = [&](auto half) {
      constexpr int L0 = decltype(half)::value * R0;
      constexpr int NR = decltype(half)::value == 0 ? R0 : NL - R0;
      T rr[KC][NR];
      uint32_t hc[KC];
      load_rows_part<NL, NR, KC, T>(rr, p.pinv, Np, NE1, 0, L0, io);
      load_pos<KC>(hc, rl, lrow, NE1, 0, io2, self);
      if constexpr (L0 == 0) __syncthreads();
      T acc[NR][VB];
#pragma unroll
      for (int l = 0; l < NR; ++l)
#pragma unroll
        for (int v = 0; v < VB; ++v) acc[l][v] = T(0);
      fma_chunk<NR, VB, KC, T>(acc, rr, hc, lq, self);
      for (int k0 = KC; k0 < NE1; k0 += KC) {
        load_rows_part<NL, NR, KC, T>(rr, p.pinv, Np, NE1, k0, L0, io);
        load_pos<KC>(hc, rl, lrow, NE1, k0, io2, self);
        fma_chunk<NR, VB, KC, T>(acc, rr, hc, lq, self);
      }
      if (valid) {
#pragma unroll
        for (int v = 0; v < VB; ++v) {
          const rsrc_t ro = make_rsrc(p.out + (int64_t)(p.v0 + v) * NB * qs, NB * crow);
#pragma unroll
          for (int l = 0; l < NR; ++l) bst_keep(ro, acc[l][v], io, (uint32_t)(1 + L0 + l) * crow);
        }
      }
    };
    pass(std::integral_constant<int, 0>{});
    pass(std::integral_constant<int, 1>{});
    T lam[NS + 1];
    const T inv_l0 = cell_weights<NS, T>(p, mask, lam);
    if (valid) {
      T bv[NS][D][D];
      load_binv<D, T>(p.binv, Np, io, bv);
      const T* sv = lq + self * VB;
#pragma unroll
      for (int v = 0; v < VB; ++v) {
        const T qi = sv[v];
        T dqs[NS][D];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int a = 0; a < D; ++a) dqs[s][a] = lq[sl[s][a] * VB + v] - qi;
        const rsrc_t ro = make_rsrc(p.out + (int64_t)(p.v0 + v) * NB * qs, NB * crow);
        T po[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) po[l] = bld<T>(ro, io, (uint32_t)(1 + l) * crow);
        finish_variable<D, M, T, false>(p, io, v, qi, po, lam, inv_l0, dqs, bv, nullptr);
      }
    }
  }
}

template <int D, int M, int VB, int KC, int HU, typename T, bool PTS = false>
__global__ __launch_bounds__(kHaloBlock) void reconstruct_halo_kernel(KParams<T> p, CWENO_ARRAY_PARAMS(T)) {
  CWENO_BIND_ARRAYS(p);
  extern __shared__ __align__(16) unsigned char halo_raw[];
  halo_block<D, M, VB, KC, HU, T, PTS>(p, xcd_block(blockIdx.x, gridDim.x), reinterpret_cast<T*>(halo_raw));
}

// Work item of the batched kernel: block `block` of the mesh (and variable
// block) whose parameters are entry `entry` of the batch table.
struct BatchItem {
  int32_t entry;
  int32_t block;
};

// Batched persistent kernel: every workgroup walks the work list with stride
// gridDim.x; the parameters of each item's mesh come from a device table (read
// through the scalar cache).  All meshes of one launch share (D, M, VB) and the
// LDS size, which covers the largest of their halos.
// Copy a structure that no kernel writes, word by word through the constant
// address space (scalar loads).
template <typename S>
__device__ __forceinline__ S load_uniform(const S* ptr) {
  static_assert(sizeof(S) % 4 == 0, "word-sized structure");
  S out;
  const __attribute__((address_space(4))) uint32_t* src = (const __attribute__((address_space(4))) uint32_t*)ptr;
  uint32_t* dst = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(S) / 4); ++k) dst[k] = src[k];
  return out;
}

template <int D, int M, int VB, int KC, int HU, typename T>
__global__ __launch_bounds__(kHaloBlock) void reconstruct_batch_kernel(const KParams<T>* table,
                                                                       const BatchItem* items, int n_items) {
  extern __shared__ __align__(16) unsigned char halo_raw[];
  T* const lq = reinterpret_cast<T*>(halo_raw);
  for (int it = (int)blockIdx.x; it < n_items; it += (int)gridDim.x) {
    const BatchItem w = load_uniform(items + it);
    const KParams<T> p = load_uniform(table + w.entry);
    halo_block<D, M, VB, KC, HU, T>(p, w.block, lq);
    __syncthreads();   // the next item overwrites the halo
  }
}

}  // namespace cweno
