// Classical unstructured WENO reconstruction kernel (gfx950, FP64): the
// scheme the paper compares CWENO with.  1 + 2(d+1) stencils -- central,
// forward and reverse cone sectors -- each of n_e cells and each giving a
// degree-M polynomial by its own stored least-squares pseudo-inverse (as for
// P_opt, eq. CWENO:Popt: p_0 = Q_i, p_{1..} = pinv_j (Q - Q_i)); indicators
// with the universal Sigma; omega~_j = lambda_j / (sigma_j + eps)^r;
// w = sum_j omega~_j P_j / sum_j omega~_j (eqs. weights, weights2).
//
// A workgroup takes kWenoBlockCells consecutive cells with a group of G = 1,
// 2, 4 or 8 lanes per cell, each lane reconstructing VB of the pass's
// variables.  It first copies the averages of its halo -- the sorted unique
// cells its stencils reference, listed on the host -- for every variable of
// the pass into LDS, then reads every stencil difference from LDS through
// 16-bit halo positions: the 1 + 2(d+1) stencils of a cell overlap, and
// neighbouring cells share most of them, so each average comes from HBM once
// per block.  Every stencil's polynomial is needed whole before its weight is
// known, so a lane keeps the polynomial being formed and the weighted running
// sum: 2 (nb-1) VB accumulators, which limits VB to 4 / 2 / 1 for nb-1 up to
// 9 / 19 / 34.  Lane s of a group loads entries s, s + G, ... of each
// operator row (a wave's load instruction returns 64 distinct values; when
// every lane of a group loaded every entry, the duplicates set the time) and
// the group shares them by lane broadcasts; operator rows stream with a
// non-temporal policy, tiled so that a row's entries for 16 cells are one
// contiguous run.  The rows of a stencil go in chunks of KC,
// double-buffered: the halo positions and operator entries of the next chunk
// are requested before the current one is used, so that a wave keeps up to
// 2 KC rows of loads in flight instead of waiting a memory round trip per row
// (the block halos hold about 13 cells per cell, so LDS allows only a few
// waves per SIMD and each must carry many loads).
//
// LDS layout: [halo cell][variable of the pass], the variables of a cell
// together.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mesh.hpp"
#include "reconstruct_kernel.hpp"
#include "weno.hpp"

namespace cweno {

// f(std::integral_constant<int, I>) for I = 0 .. N-1 (compile-time indices).
template <int I, int N>
struct StaticForW {
  template <typename F>
  __device__ __forceinline__ static void run(F& f) {
    f(std::integral_constant<int, I>{});
    StaticForW<I + 1, N>::run(f);
  }
};
template <int N>
struct StaticForW<N, N> {
  template <typename F>
  __device__ __forceinline__ static void run(F&) {}
};

// Value of x in lane SRC of this lane's group of G consecutive lanes (G = 1,
// 2, 4 or 8; a group never crosses a DPP row): quad permutations for pairs
// and quads; for 8 lanes the quad holding lane SRC is then copied to the
// group's other quad by a 4-lane row shift written to that quad's banks.
template <int G, int SRC>
__device__ __forceinline__ double group_bcast(double x) {
  static_assert(SRC >= 0 && SRC < G, "lane of the group");
  auto dpp = [](double y, auto ctrl, auto banks, double old) {
    constexpr int C = decltype(ctrl)::value, B = decltype(banks)::value;
    const uint64_t u = __builtin_bit_cast(uint64_t, y), o = __builtin_bit_cast(uint64_t, old);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u, C, 0xF, B, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32), C, 0xF, B, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  };
  // a quad permutation writes every lane from a lane of its own quad: no
  // old value to keep, so none is copied into the destination first
  auto perm = [](double y, auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    const uint64_t u = __builtin_bit_cast(uint64_t, y);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, C, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), C, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
  };
  if constexpr (G == 1) {
    return x;
  } else if constexpr (G == 2) {
    return perm(x, std::integral_constant<int, SRC | SRC << 2 | (2 + SRC) << 4 | (2 + SRC) << 6>{});
  } else if constexpr (G == 4) {
    return perm(x, std::integral_constant<int, SRC * 0x55>{});
  } else {
    static_assert(G == 8, "groups of 1, 2, 4 or 8 lanes");
    const double a = perm(x, std::integral_constant<int, (SRC % 4) * 0x55>{});
    if constexpr (SRC < 4)
      return dpp(a, std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xA>{}, a);   // row_shr:4
    else
      return dpp(a, std::integral_constant<int, 0x104>{}, std::integral_constant<int, 0x5>{}, a);   // row_shl:4
  }
}

template <int D, int M, int VB, int G>
__global__ __launch_bounds__(kWenoBlockCells * kWenoMaxGroup) void weno_kernel(WParams p) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  constexpr int NT = (NL + G - 1) / G;                  // entries of a row each lane of a group loads
  constexpr int KC = weno_kc(D, M, VB, G);
  constexpr int KB = KC > 0 ? KC : 1;
  constexpr int T = kWenoTile;
  extern __shared__ double lq[];
  const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
  const int nvp = p.v1 - p.v0;
  const int64_t nc = p.nc, Np = p.Np;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);

  // stage the block's halo, cell-fastest so that runs of consecutive cells
  // read consecutive addresses; SU cells per thread at a time, so that each
  // round is two memory round trips (positions, then averages)
  {
    constexpr int VMAX = VB * G;
    constexpr int SU = VMAX >= 16 ? 1 : 32 / VMAX < 4 ? 32 / VMAX : 4;
    const int h0 = p.hoff[b], hn = p.hoff[b + 1] - h0;
    for (int hb = tid; hb < hn; hb += SU * nthr) {
      int64_t c[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) c[u] = hb + u * nthr < hn ? p.halo[h0 + hb + u * nthr] : -1;
      double x[SU][VMAX];
#pragma unroll
      for (int u = 0; u < SU; ++u)
#pragma unroll
        for (int v = 0; v < VMAX; ++v)
          if (v < nvp && c[u] >= 0) x[u][v] = p.q[(int64_t)(p.v0 + v) * nc + c[u]];
#pragma unroll
      for (int u = 0; u < SU; ++u)
#pragma unroll
        for (int v = 0; v < VMAX; ++v)
          if (v < nvp && c[u] >= 0) lq[(hb + u * nthr) * nvp + v] = x[u][v];
    }
  }
  __syncthreads();

  // every lane of a group stays to the end: it loads its share of each row
  // for the others; a cell past the mesh works on the last cell and stores
  // nothing, a lane without variables repeats the pass's last one
  const int cw = tid / G, sub = tid - cw * G;
  const int64_t i = b * kWenoBlockCells + cw;
  const bool live = i < nc;
  const int64_t ic = live ? i : nc - 1;
  const int vofs = sub * VB;                            // this lane's first variable within the pass
  const int nvl = min(VB, nvp - vofs);                  // and how many it owns (may be none)
  const int NE1 = p.NE1, n_s = p.n_s;
  const uint16_t* li = p.lidx + ic;
  int vv[VB];                                           // LDS column of each variable
#pragma unroll
  for (int v = 0; v < VB; ++v) vv[v] = min(vofs + v, nvp - 1);
  const double* ls = lq + (int)li[(int64_t)n_s * NE1 * Np] * nvp;
  double qi[VB];
#pragma unroll
  for (int v = 0; v < VB; ++v) qi[v] = ls[vv[v]];
  const unsigned am = p.alive[ic];
  double lsum = 0.0;
  for (int j = 0; j < n_s; ++j)
    if ((am >> j) & 1u) lsum += j == 0 ? p.lam0 : p.lams;
  double wn[NL][VB], ws[VB];
#pragma unroll
  for (int v = 0; v < VB; ++v) {
    ws[v] = 0.0;
#pragma unroll
    for (int l = 0; l < NL; ++l) wn[l][v] = 0.0;
  }
  for (int j = 0; j < n_s; ++j) {
    if (!((am >> j) & 1u)) continue;                    // the same for every lane of a group
    const double lj = (j == 0 ? p.lam0 : p.lams) / lsum;
    double acc[NL][VB];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int v = 0; v < VB; ++v) acc[l][v] = 0.0;
    const double* pj = p.pinv + (int64_t)j * NE1 * NL * Np + (ic / T) * NL * T + ic % T;
    const uint16_t* lj16 = li + (int64_t)j * NE1 * Np;
    // lane sub of a group loads entries sub, sub + G, ... of a row (distinct
    // addresses across the group) and the group shares them by lane
    // broadcasts; chunk c+1's requests go out before chunk c is used (two
    // chunks of rows in registers), so that a wave always has loads in flight
    int hp[2][KB];
    double r[2][KB][NT];
    auto request = [&](int bf, int k0) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int k = min(k0 + u, NE1 - 1);             // past the stencil: its last row again, not used
        hp[bf][u] = lj16[(int64_t)k * Np];
        const double* pk = pj + (int64_t)k * NL * Np;
#pragma unroll
        for (int t = 0; t < NT; ++t) r[bf][u][t] = __builtin_nontemporal_load(pk + min(sub + G * t, NL - 1) * T);
      }
    };
    auto consume = [&](int bf, int k0) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        if (k0 + u >= NE1) break;
        const double* lh = lq + hp[bf][u] * nvp;
        double dq[VB];
#pragma unroll
        for (int v = 0; v < VB; ++v) dq[v] = lh[vv[v]] - qi[v];
        auto entry = [&](auto lc) {
          constexpr int l = decltype(lc)::value;
          const double x = group_bcast<G, l % G>(r[bf][u][l / G]);
#pragma unroll
          for (int v = 0; v < VB; ++v) acc[l][v] = fma(x, dq[v], acc[l][v]);
        };
        StaticForW<0, NL>::run(entry);
      }
    };
    if constexpr (KC > 0) {
      request(0, 0);
      for (int k0 = 0; k0 < NE1; k0 += 2 * KC) {
        // the barriers keep each chunk's requests ahead of the other's uses
        // (the scheduler would sink every row's loads to its multiply-adds)
        if (k0 + KC < NE1) request(1, k0 + KC);
        __builtin_amdgcn_sched_barrier(0);
        consume(0, k0);
        if (k0 + 2 * KC < NE1) request(0, k0 + 2 * KC);
        __builtin_amdgcn_sched_barrier(0);
        if (k0 + KC < NE1) consume(1, k0 + KC);
      }
    } else {
      for (int k = 0; k < NE1; ++k) {
        request(0, k);
        consume(0, k);
      }
    }
#pragma unroll
    for (int v = 0; v < VB; ++v) {
      double pv[NL];
#pragma unroll
      for (int l = 0; l < NL; ++l) pv[l] = acc[l][v];
      double m[1] = {quad_form<D, M, double>(pv) + p.eps};
      powi<1, double>(m, p.r);
      const double wt = lj / m[0];
      ws[v] += wt;
#pragma unroll
      for (int l = 0; l < NL; ++l) wn[l][v] = fma(wt, acc[l][v], wn[l][v]);
    }
  }
  if (!live) return;
#pragma unroll
  for (int v = 0; v < VB; ++v) {
    if (v >= nvl) break;
    double* o = p.out + (int64_t)(p.v0 + vofs + v) * NB * nc + i;
    o[0] = qi[v];
    const double iw = 1.0 / ws[v];
#pragma unroll
    for (int l = 0; l < NL; ++l) __builtin_nontemporal_store(wn[l][v] * iw, o + (int64_t)(l + 1) * nc);
  }
}

namespace {

template <int D, int M>
hipError_t launch_dm(const WParams& p, int vb, int max_halo, hipStream_t s) {
  const int nvp = p.v1 - p.v0;
  if ((p.G != 1 && p.G != 2 && p.G != 4 && p.G != 8) || nvp < 1 || nvp > p.G * vb) return hipErrorInvalidValue;
  const size_t lds = (size_t)max_halo * (size_t)nvp * sizeof(double);
  if (lds > kWenoMaxLds) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((p.nc + kWenoBlockCells - 1) / kWenoBlockCells);
  const unsigned threads = (unsigned)(kWenoBlockCells * p.G);
  auto go = [&](auto vbc, auto gc) -> hipError_t {
    constexpr int V = decltype(vbc)::value, G = decltype(gc)::value;
    if constexpr (V <= weno_vb_max(D, M)) {
      hipLaunchKernelGGL((weno_kernel<D, M, V, G>), dim3(blocks), dim3(threads), lds, s, p);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  };
  auto by_g = [&](auto vbc) -> hipError_t {
    switch (p.G) {
      case 1: return go(vbc, std::integral_constant<int, 1>{});
      case 2: return go(vbc, std::integral_constant<int, 2>{});
      case 4: return go(vbc, std::integral_constant<int, 4>{});
      case 8: return go(vbc, std::integral_constant<int, 8>{});
    }
    return hipErrorInvalidValue;
  };
  switch (vb) {
    case 1: return by_g(std::integral_constant<int, 1>{});
    case 2: return by_g(std::integral_constant<int, 2>{});
    case 3: return by_g(std::integral_constant<int, 3>{});
    case 4: return by_g(std::integral_constant<int, 4>{});
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_weno(int d, int M, const WParams& p, int vb, int max_halo, hipStream_t s) {
  switch (d * 10 + M) {
    case 21: return launch_dm<2, 1>(p, vb, max_halo, s);
    case 22: return launch_dm<2, 2>(p, vb, max_halo, s);
    case 23: return launch_dm<2, 3>(p, vb, max_halo, s);
    case 24: return launch_dm<2, 4>(p, vb, max_halo, s);
    case 31: return launch_dm<3, 1>(p, vb, max_halo, s);
    case 32: return launch_dm<3, 2>(p, vb, max_halo, s);
    case 33: return launch_dm<3, 3>(p, vb, max_halo, s);
    case 34: return launch_dm<3, 4>(p, vb, max_halo, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace cweno
