// Producer/consumer variant of the CWENO reconstruction kernel (gfx950).
//
// Same arithmetic as reconstruct_kernel (one lane per cell; each P_opt row a
// FMA chain over the stencil in order k = 0, 1, ...; identical epilogue).
// What changes is who waits for which memory:
//
//  * One producer wavefront per workgroup streams, for stencil entry k, the
//    operator rows of the workgroup's C = 64 * NCW cells and the gather-index
//    row of entry k + P from HBM into registers, DP entries ahead, and writes
//    entry k + 1 into the LDS stage (k + 1) mod 2 while entry k is consumed.
//    Its loads are all of one kind, so the compiler's wait counts are exact
//    and it only ever waits for the loads of the entry it writes next.
//  * NCW consumer wavefronts read the operator rows of entry k from LDS and
//    gather the neighbour averages of entry k + P (indices from LDS) into
//    registers, P entries before they are needed.  Their load queue holds only
//    those gathers, which hit L2.
//  * An LDS-only barrier (lgkmcnt(0); s_barrier) separates the entries; it
//    does not drain either queue of vector-memory loads.
//
// The workgroup covers cells c0 .. c0 + C - 1; consumer wavefront w owns cells
// c0 + 64 w + lane.  Lanes past the last cell compute on their own index and
// store nothing.
#pragma once

#include "reconstruct_kernel.hpp"

namespace cweno {

__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int NL, int NCW, typename T>
struct PcShape {
  static constexpr int C = 64 * NCW;                          // cells per workgroup
  static constexpr int ROW16 = C * (int)sizeof(T) / 16;       // 16-byte chunks per operator row
  static constexpr int NR16 = NL * ROW16;                     // operator chunks per entry
  static constexpr int NG16 = C / 4;                          // gather-index chunks per entry
  static constexpr int CH = (NR16 + NG16 + 63) / 64;          // chunks per producer lane
  static constexpr int STAGE = (NR16 + NG16) * 16;            // bytes per LDS stage
};

template <int D, int M, int NCW, typename T>
__host__ __device__ constexpr int pc_lds_bytes() {
  return 2 * PcShape<nbasis_c(M, D) - 1, NCW, T>::STAGE;
}

// Producer: load the chunks of entry k (operator rows k, index row k + P).
template <int NL, int NCW, int P, typename T, int CH>
__device__ __forceinline__ void pc_load(uint4 (&buf)[CH], const KParams<T>& p, int64_t c0, int lane, int k) {
  using S = PcShape<NL, NCW, T>;
  constexpr int EPL = 16 / (int)sizeof(T);
  const int64_t Np = p.Np;
  static_assert(CH == S::CH, "chunk count");
#pragma unroll
  for (int m = 0; m < S::CH; ++m) {
    const int t = lane + 64 * m;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (t < S::NR16) {
      const int row = t / S::ROW16, col = t % S::ROW16;
      const int64_t cell = c0 + (int64_t)col * EPL;
      if (cell < Np)
        v = *reinterpret_cast<const uint4*>(p.pinv + ((int64_t)k * NL + row) * Np + cell);
    } else if (t < S::NR16 + S::NG16) {
      const int g = t - S::NR16;
      const int64_t cell = c0 + 4 * (int64_t)g;
      if (k + P < p.NE1 && cell < Np)
        v = *reinterpret_cast<const uint4*>(p.gidx + (int64_t)(k + P) * Np + cell);
    }
    buf[m] = v;
  }
}

template <int NL, int NCW, typename T, int CH>
__device__ __forceinline__ void pc_store(unsigned char* stage, const uint4 (&buf)[CH], int lane) {
  using S = PcShape<NL, NCW, T>;
  static_assert(CH == S::CH, "chunk count");
#pragma unroll
  for (int m = 0; m < S::CH; ++m) {
    const int t = lane + 64 * m;
    if (t < S::NR16 + S::NG16) *reinterpret_cast<uint4*>(stage + t * 16) = buf[m];
  }
}

template <int D, int M, int VB, int NCW, int DP, int P, typename T>
__global__ __launch_bounds__(64 * (NCW + 1)) void reconstruct_pc_kernel(KParams<T> p) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NS_ = D + 1;
  using S = PcShape<NL, NCW, T>;
  static_assert(DP >= 2 && P >= 1, "pipeline depths");
  __shared__ __align__(16) unsigned char lds[2 * S::STAGE];

  const int lane = (int)threadIdx.x & 63;
  const int w = (int)threadIdx.x >> 6;
  const int64_t c0 = xcd_block(blockIdx.x, gridDim.x) * S::C;
  const int NE1 = p.NE1;

  if (w == NCW) {
    // ---------------------------------------------------------------- producer
    uint4 buf[DP][S::CH];
#pragma unroll
    for (int s = 0; s < DP; ++s)
      if (s < NE1) pc_load<NL, NCW, P, T, S::CH>(buf[s], p, c0, lane, s);
    pc_store<NL, NCW, T, S::CH>(lds, buf[0], lane);
    lds_barrier();
    for (int k0 = 0; k0 < NE1; k0 += DP) {
#pragma unroll
      for (int u = 0; u < DP; ++u) {
        const int k = k0 + u;
        if (k < NE1) {
          if (k + DP < NE1) pc_load<NL, NCW, P, T, S::CH>(buf[u], p, c0, lane, k + DP);
          if (k + 1 < NE1) pc_store<NL, NCW, T, S::CH>(lds + ((k + 1) & 1) * S::STAGE, buf[(u + 1) % DP], lane);
          lds_barrier();
        }
      }
    }
    return;
  }

  // ---------------------------------------------------------------- consumers
  const int64_t i = c0 + 64 * w + lane;
  const bool valid = i < p.nc;
  const int64_t ic = valid ? i : p.nc - 1;
  const int64_t Np = p.Np, qs = p.nc;
  const T* __restrict__ q = p.q + (int64_t)p.v0 * qs;
  const uint32_t io = (uint32_t)ic * (uint32_t)sizeof(T);
  const uint32_t io4 = (uint32_t)ic * 4u;
  const int slot = 64 * w + lane;                      // this cell's column in a stage

  int32_t sj[NS_][D];
#pragma unroll
  for (int s = 0; s < NS_; ++s)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const uint32_t pos = ldo(p.secpos + (s * D + a) * Np, (uint32_t)ic);
      sj[s][a] = ldo(p.gidx + (int64_t)pos * Np, io4);
    }
  const unsigned mask = ldo(p.mask, (uint32_t)ic);

  T qi[VB];
#pragma unroll
  for (int v = 0; v < VB; ++v) qi[v] = ldo(q + v * qs, io);

  // neighbour averages of entry k live in gb[k mod (P+1)]; entries 0..P-1 now
  T gb[P + 1][VB];
#pragma unroll
  for (int t = 0; t < P; ++t) {
    const uint32_t j = t < NE1 ? (uint32_t)ldo(p.gidx + (int64_t)t * Np, io4) : (uint32_t)ic;
#pragma unroll
    for (int v = 0; v < VB; ++v) gb[t][v] = ldo(q + v * qs, j * (uint32_t)sizeof(T));
  }

  T acc[NL][VB];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int v = 0; v < VB; ++v) acc[l][v] = T(0);

  lds_barrier();
  for (int k0 = 0; k0 < NE1; k0 += P + 1) {
#pragma unroll
    for (int u = 0; u <= P; ++u) {
      const int k = k0 + u;
      if (k < NE1) {
        const unsigned char* st = lds + (k & 1) * S::STAGE;
        if (k + P < NE1) {
          const uint32_t jl = *reinterpret_cast<const uint32_t*>(st + NL * S::C * (int)sizeof(T) + slot * 4);
          const uint32_t j = valid ? jl : (uint32_t)ic;
#pragma unroll
          for (int v = 0; v < VB; ++v) gb[(u + P) % (P + 1)][v] = ldo(q + v * qs, j * (uint32_t)sizeof(T));
        }
        const T* rows = reinterpret_cast<const T*>(st);
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const T r = rows[l * S::C + slot];
#pragma unroll
          for (int v = 0; v < VB; ++v) acc[l][v] = fma(r, gb[u][v] - qi[v], acc[l][v]);
        }
        lds_barrier();
      }
    }
  }

  // Linear weights of this cell: dropped sectors get 0, the rest renormalised.
  T lam[NS_ + 1];
  T lsum = p.lam[0];
  lam[0] = p.lam[0];
#pragma unroll
  for (int s = 0; s < NS_; ++s) {
    lam[s + 1] = ((mask >> s) & 1u) ? p.lam[s + 1] : T(0);
    lsum += lam[s + 1];
  }
#pragma unroll
  for (int s = 0; s <= NS_; ++s) lam[s] /= lsum;
  const T inv_l0 = T(1) / lam[0];
  if (!valid) return;
#pragma unroll
  for (int v = 0; v < VB; ++v) {
    T dqs[NS_][D];
    sector_dq_global<D, T>(p, v, qi[v], sj, dqs);
    finish_variable<D, M, T>(p, i, v, qi[v], [&](int l) { return acc[l][v]; }, lam, inv_l0, dqs);
  }
}

}  // namespace cweno
