// Launcher of the classical unstructured WENO kernel (the comparison scheme).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "reconstruct_kernel.hpp"

namespace cweno {

// Cells per workgroup of the WENO kernel, the block size of its host halos.
constexpr int kWenoBlockCells = 64;

struct WParams {
  const double* q;        // [nv][nc]
  double* out;            // [nv][NB][nc]
  const double* pinv;     // [(j * NE1 + k) * NL + l][Np]
  const uint16_t* lidx;   // [j * NE1 + k][Np] halo position of stencil entry k+1; row n_s NE1: the cell
  const int32_t* halo;    // concatenated block halos (sorted unique cells)
  const int32_t* hoff;    // [blocks + 1] offsets into halo
  const uint16_t* alive;  // [Np] bit j: stencil j kept
  double lam0, lams, eps; // linear weight of the central stencil and of each sector stencil
  int64_t nc, Np;
  int NE1, n_s, r;
  int v0, v1;             // the pass reconstructs variables v0 .. v1-1
  int G;                  // lanes per cell (1 .. kWenoMaxGroup), VB variables each
};

// Variables per lane: the polynomial being formed and the weighted sum take
// 2 (nb-1) VB doubles per lane.
__host__ __device__ constexpr int weno_vb_max(int D, int M) {
  return nbasis_c(M, D) - 1 <= 9 ? 4 : nbasis_c(M, D) - 1 <= 19 ? 2 : 1;
}
constexpr int kWenoMaxGroup = 8;
// LDS a workgroup may stage (the dynamic limit that needs no attribute).
constexpr size_t kWenoMaxLds = 65536;

// One pass: variables v0 .. v1-1 with G lanes per cell, vb variables each;
// max_halo is the mesh's longest block halo (LDS = max_halo (v1-v0) doubles).
hipError_t launch_weno(int d, int M, const WParams& p, int vb, int max_halo, hipStream_t s);

}  // namespace cweno
