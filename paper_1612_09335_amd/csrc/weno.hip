// Classical unstructured WENO reconstruction kernel (gfx950, FP64): the
// scheme the paper compares CWENO with.  1 + 2(d+1) stencils -- central,
// forward and reverse cone sectors -- each of n_e cells and each giving a
// degree-M polynomial by its own stored least-squares pseudo-inverse (as for
// P_opt, eq. CWENO:Popt: p_0 = Q_i, p_{1..} = pinv_j (Q - Q_i)); indicators
// with the universal Sigma; omega~_j = lambda_j / (sigma_j + eps)^r;
// w = sum_j omega~_j P_j / sum_j omega~_j (eqs. weights, weights2).
//
// A workgroup takes kWenoBlockCells consecutive cells with a group of G lanes
// per cell (G <= 8), each lane reconstructing VB of the pass's variables.  It
// first copies the averages of its halo -- the sorted unique cells its
// stencils reference, listed on the host -- for every variable of the pass
// into LDS, then reads every stencil difference from LDS through 16-bit
// halo positions: the 1 + 2(d+1) stencils of a cell overlap, and neighbouring
// cells share most of them, so each average comes from HBM once per block.
// Every stencil's polynomial is needed whole before its weight is known, so a
// lane keeps the polynomial being formed and the weighted running sum:
// 2 (nb-1) VB accumulators, which limits VB to 4 / 2 / 1 for nb-1 up to
// 9 / 19 / 34.  The lanes of a group load the same operator entries in the
// same instruction, so the wave fetches each entry once per pass; operator
// rows stream with a non-temporal policy.
//
// LDS layout: [halo cell][variable of the pass], the variables of a cell
// together.
#include <hip/hip_runtime.h>

#include "mesh.hpp"
#include "reconstruct_kernel.hpp"
#include "weno.hpp"

namespace cweno {

template <int D, int M, int VB>
__global__ __launch_bounds__(kWenoBlockCells * kWenoMaxGroup) void weno_kernel(WParams p) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  extern __shared__ double lq[];
  const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
  const int G = p.G, nvp = p.v1 - p.v0;
  const int64_t nc = p.nc, Np = p.Np;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);

  // stage the block's halo, cell-fastest so that runs of consecutive cells
  // read consecutive addresses
  const int h0 = p.hoff[b], hn = p.hoff[b + 1] - h0;
  for (int hc = tid; hc < hn; hc += nthr) {
    const int64_t c = p.halo[h0 + hc];
    const double* qc = p.q + (int64_t)p.v0 * nc + c;
    for (int v = 0; v < nvp; ++v) lq[hc * nvp + v] = qc[(int64_t)v * nc];
  }
  __syncthreads();

  const int cw = tid / G, sub = tid - cw * G;
  const int64_t i = b * kWenoBlockCells + cw;
  if (i >= nc) return;
  const int vofs = sub * VB;                            // this lane's first variable within the pass
  const int nvl = min(VB, nvp - vofs);                  // and how many it owns
  if (nvl <= 0) return;
  const int NE1 = p.NE1, n_s = p.n_s;
  const uint16_t* li = p.lidx + i;
  int vv[VB];                                           // LDS column of each variable (the last repeated)
#pragma unroll
  for (int v = 0; v < VB; ++v) vv[v] = vofs + min(v, nvl - 1);
  const double* ls = lq + (int)li[(int64_t)n_s * NE1 * Np] * nvp;
  double qi[VB];
#pragma unroll
  for (int v = 0; v < VB; ++v) qi[v] = ls[vv[v]];
  const unsigned am = p.alive[i];
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
    if (!((am >> j) & 1u)) continue;
    const double lj = (j == 0 ? p.lam0 : p.lams) / lsum;
    double acc[NL][VB];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int v = 0; v < VB; ++v) acc[l][v] = 0.0;
    const double* pj = p.pinv + (int64_t)j * NE1 * NL * Np + i;
    const uint16_t* lj16 = li + (int64_t)j * NE1 * Np;
    for (int k = 0; k < NE1; ++k) {
      const double* lh = lq + (int)lj16[(int64_t)k * Np] * nvp;
      double dq[VB];
#pragma unroll
      for (int v = 0; v < VB; ++v) dq[v] = lh[vv[v]] - qi[v];
      const double* pk = pj + (int64_t)k * NL * Np;
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const double r = __builtin_nontemporal_load(pk + (int64_t)l * Np);
#pragma unroll
        for (int v = 0; v < VB; ++v) acc[l][v] = fma(r, dq[v], acc[l][v]);
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
  if (p.G < 1 || p.G > kWenoMaxGroup || nvp < 1 || nvp > p.G * vb) return hipErrorInvalidValue;
  const size_t lds = (size_t)max_halo * (size_t)nvp * sizeof(double);
  if (lds > kWenoMaxLds) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((p.nc + kWenoBlockCells - 1) / kWenoBlockCells);
  const unsigned threads = (unsigned)(kWenoBlockCells * p.G);
  switch (vb) {
#define CWENO_WENO_VB(V)                                                                                         \
  case V:                                                                                                        \
    if constexpr (V <= weno_vb_max(D, M)) {                                                                      \
      hipLaunchKernelGGL((weno_kernel<D, M, V>), dim3(blocks), dim3(threads), lds, s, p);                         \
      return hipGetLastError();                                                                                  \
    }                                                                                                            \
    break;
    CWENO_WENO_VB(1) CWENO_WENO_VB(2) CWENO_WENO_VB(3) CWENO_WENO_VB(4)
#undef CWENO_WENO_VB
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
