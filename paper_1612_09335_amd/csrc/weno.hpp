// Launcher of the classical unstructured WENO kernel (the comparison scheme).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "reconstruct_kernel.hpp"

namespace cweno {

// Cells per workgroup of the WENO kernel, the block size of its host halos.
constexpr int kWenoBlockCells = 64;

// Operator rows on the device are tiled over kWenoTile cells: entry l of row
// k of stencil j of cell i sits at
//   (((j NE1 + k) Np / kWenoTile + i / kWenoTile) NL + l) kWenoTile + i % kWenoTile,
// so that the NL entries of one row for a tile of cells are one contiguous
// run (a wave reading a row sweeps whole runs however many lanes share a
// cell; with one plane per entry it read only 8 bytes per cell it holds from
// each plane).
constexpr int kWenoTile = 16;

struct WParams {
  const double* q;        // [nv][nc]
  double* out;            // [nv][NB][nc]
  const double* pinv;     // tiled, see above
  const uint16_t* lidx;   // [j * NE1 + k][Np] halo position of stencil entry k+1; row n_s NE1: the cell
  const int32_t* halo;    // concatenated block halos (sorted unique cells)
  const int32_t* hoff;    // [blocks + 1] offsets into halo
  const uint16_t* alive;  // [Np] bit j: stencil j kept
  double lam0, lams, eps; // linear weight of the central stencil and of each sector stencil
  int64_t nc, Np;
  int NE1, n_s, r;
  int v0, v1;             // the pass reconstructs variables v0 .. v1-1
  int G;                  // lanes per cell (1, 2, 4 or 8), VB variables each
};

// Variables per lane: the polynomial being formed and the weighted sum take
// 2 (nb-1) VB doubles per lane.
__host__ __device__ constexpr int weno_vb_max(int D, int M) {
  return nbasis_c(M, D) - 1 <= 9 ? 4 : nbasis_c(M, D) - 1 <= 19 ? 2 : 1;
}
constexpr int kWenoMaxGroup = 8;
// Stencil rows per chunk, double-buffered (2 KC rows of a lane's share of
// the operator entries, ceil((nb-1)/G) each, in registers beside the
// 2 (nb-1) VB accumulators): as many, up to 4, as keep the total within
// about 90 doubles (70 for the 34 basis functions of 3-D degree 4 or
// accumulators above 72), one row at 72, else 0 -- one row at a time, left to
// the scheduler.  The bounds are where the register allocation stops fitting
// without spills; measured on the 2-D degree-3 workload, 90 against 70 took
// 9 variables from 1.46 to 1.41 ms and 8 from 1.83 to 1.56 ms.
__host__ __device__ constexpr int weno_kc(int D, int M, int VB, int G) {
  const int nl = nbasis_c(M, D) - 1, nt = (nl + G - 1) / G, accd = 2 * nl * VB;
  const int kc = ((nl > 19 || accd > 72 ? 70 : 90) - accd) / (2 * nt);
  return kc < 0 ? 0 : kc > (accd >= 72 ? 1 : 4) ? (accd >= 72 ? 1 : 4) : kc;
}
// LDS a workgroup may stage (the dynamic limit that needs no attribute).
constexpr size_t kWenoMaxLds = 65536;

// One pass: variables v0 .. v1-1 with G lanes per cell (1, 2, 4 or 8), vb
// variables each;
// max_halo is the mesh's longest block halo (LDS = max_halo (v1-v0) doubles).
hipError_t launch_weno(int d, int M, const WParams& p, int vb, int max_halo, hipStream_t s);

}  // namespace cweno
