// Classical unstructured WENO reconstruction kernel (gfx950, FP64): the
// scheme the paper compares CWENO with.  1 + 2(d+1) stencils -- central,
// forward and reverse cone sectors -- each of n_e cells and each giving a
// degree-M polynomial by its own stored least-squares pseudo-inverse (as for
// P_opt, eq. CWENO:Popt: p_0 = Q_i, p_{1..} = pinv_j (Q - Q_i)); indicators
// with the universal Sigma; omega~_j = lambda_j / (sigma_j + eps)^r;
// w = sum_j omega~_j P_j / sum_j omega~_j (eqs. weights, weights2).
//
// One lane per cell, VB variables per pass.  Every stencil's polynomial is
// needed whole before its weight is known, so a pass keeps the polynomial
// being formed and the weighted running sum: 2 (nb-1) VB accumulators, which
// limits VB to 4 / 2 / 1 for nb-1 up to 9 / 19 / 34.  Operator rows stream
// once per pass with a non-temporal policy; neighbour averages are gathered.
#include <hip/hip_runtime.h>

#include "mesh.hpp"
#include "reconstruct_kernel.hpp"
#include "weno.hpp"

namespace cweno {

template <int D, int M, int VB>
__global__ __launch_bounds__(kThreads) void weno_kernel(WParams p, const double* __restrict__ q,
                                                        double* __restrict__ out, const double* __restrict__ pinv,
                                                        const int32_t* __restrict__ gidx,
                                                        const uint16_t* __restrict__ alive) {
  constexpr int NB = nbasis_c(M, D);
  constexpr int NL = NB - 1;
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (i >= p.nc) return;
  const int64_t nc = p.nc, Np = p.Np;
  const int NE1 = p.NE1, n_s = p.n_s;
  const double* qb = q + (int64_t)p.v0 * nc;
  double qi[VB];
#pragma unroll
  for (int v = 0; v < VB; ++v) qi[v] = qb[v * nc + i];
  const unsigned am = alive[i];
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
    const double* pj = pinv + (int64_t)j * NE1 * NL * Np + i;
    const int32_t* gj = gidx + (int64_t)j * NE1 * Np + i;
    for (int k = 0; k < NE1; ++k) {
      const int64_t c = gj[(int64_t)k * Np];
      double dq[VB];
#pragma unroll
      for (int v = 0; v < VB; ++v) dq[v] = qb[v * nc + c] - qi[v];
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
    double* o = out + (int64_t)(p.v0 + v) * NB * nc + i;
    o[0] = qi[v];
    const double iw = 1.0 / ws[v];
#pragma unroll
    for (int l = 0; l < NL; ++l) __builtin_nontemporal_store(wn[l][v] * iw, o + (int64_t)(l + 1) * nc);
  }
}

namespace {

template <int D, int M>
hipError_t launch_dm(const WParams& p, int vb, hipStream_t s) {
  const unsigned blocks = (unsigned)((p.nc + kThreads - 1) / kThreads);
  switch (vb) {
#define CWENO_WENO_VB(V)                                                                                         \
  case V:                                                                                                        \
    if constexpr (V <= weno_vb_max(D, M)) {                                                                      \
      hipLaunchKernelGGL((weno_kernel<D, M, V>), dim3(blocks), dim3(kThreads), 0, s, p, p.q, p.out, p.pinv,      \
                         p.gidx, p.alive);                                                                       \
      return hipGetLastError();                                                                                  \
    }                                                                                                            \
    break;
    CWENO_WENO_VB(1) CWENO_WENO_VB(2) CWENO_WENO_VB(3) CWENO_WENO_VB(4)
#undef CWENO_WENO_VB
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_weno(int d, int M, const WParams& p, int vb, hipStream_t s) {
  switch (d * 10 + M) {
    case 21: return launch_dm<2, 1>(p, vb, s);
    case 22: return launch_dm<2, 2>(p, vb, s);
    case 23: return launch_dm<2, 3>(p, vb, s);
    case 24: return launch_dm<2, 4>(p, vb, s);
    case 31: return launch_dm<3, 1>(p, vb, s);
    case 32: return launch_dm<3, 2>(p, vb, s);
    case 33: return launch_dm<3, 3>(p, vb, s);
    case 34: return launch_dm<3, 4>(p, vb, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace cweno
