// Launcher of the classical unstructured WENO kernel (the comparison scheme).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "reconstruct_kernel.hpp"

namespace cweno {

struct WParams {
  const double* q;        // [nv][nc]
  double* out;            // [nv][NB][nc]
  const double* pinv;     // [(j * NE1 + k) * NL + l][Np]
  const int32_t* gidx;    // [j * NE1 + k][Np]
  const uint16_t* alive;  // [Np] bit j: stencil j kept
  double lam0, lams, eps; // linear weight of the central stencil and of each sector stencil
  int64_t nc, Np;
  int NE1, n_s, v0, r;
};

// Variables per pass: the polynomial being formed and the weighted sum take
// 2 (nb-1) VB doubles per lane.
__host__ __device__ constexpr int weno_vb_max(int D, int M) {
  return nbasis_c(M, D) - 1 <= 9 ? 4 : nbasis_c(M, D) - 1 <= 19 ? 2 : 1;
}

hipError_t launch_weno(int d, int M, const WParams& p, int vb, hipStream_t s);

}  // namespace cweno
