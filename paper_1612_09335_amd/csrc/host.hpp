// Host-side (CPU, FP64) precompute of the CWENO reconstruction operators.
//
// Everything here runs once per mesh (Sec. 2.1: on fixed meshes the stencils
// and inverted least-squares matrices are computed in a pre-processing stage
// and stored).  The device kernels only apply what is built here.
#pragma once

#include <algorithm>
#include <cstdint>
#include <exception>
#include <mutex>
#include <stdexcept>
#include <thread>
#include <string>
#include <vector>

#include "cweno.h"

namespace cweno {

struct Error : std::runtime_error {
  cweno_status code;
  Error(cweno_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Basis size of eq. cwenoM: (1/d!) prod_{l=1..d} (M + l).
int n_basis(int M, int d);

// Run f(begin, end) over [0, n) split across the hardware threads; the first
// exception thrown by any chunk is rethrown on the calling thread.
template <class F>
void parallel_for(int64_t n, F&& f) {
  int nt = (int)std::max(1u, std::thread::hardware_concurrency());
  if (nt > 64) nt = 64;
  if (n < 2048 || nt == 1) { f(int64_t(0), n); return; }
  std::vector<std::thread> th;
  std::exception_ptr err;
  std::mutex mu;
  int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([&, b, e] {
      try { f(b, e); } catch (...) { std::lock_guard<std::mutex> g(mu); if (!err) err = std::current_exception(); }
    });
  }
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

struct MeshInput {
  int d = 2;
  int64_t nv = 0;
  const double* V = nullptr;     // [nv][d]
  int64_t nc = 0;
  const int32_t* C = nullptr;    // [nc][d+1]
  double box[3] = {0, 0, 0};
};

// Unwrapped per-cell geometry (minimum image around each cell's vertex 0).
struct Geometry {
  int d = 2;
  int64_t nc = 0;
  double box[3] = {0, 0, 0};
  std::vector<double> X;    // [nc][d+1][d] unwrapped vertices
  std::vector<double> cen;  // [nc][d] barycentres
};

struct Stencils {
  int n_e = 0;
  std::vector<int32_t> central;  // [nc][n_e], cell first
  std::vector<int32_t> sectors;  // [nc][d+1][d+1], cell first; -1 row = unfillable
};

// Per-cell operators in the device layout: structure of arrays, one row per
// operator entry, the cell index fastest, row stride Np (>= nc, multiple of 64).
struct Operators {
  int d = 2, M = 1, nb = 0, n_e = 0, G = 0;
  int64_t nc = 0, Np = 0;
  std::vector<double> pinv;     // [(n_e-1)*(nb-1)][Np], row (k, l) = k*(nb-1)+l
  std::vector<double> binv;     // [(d+1)*d*d][Np], row (s, l, a)
  std::vector<int32_t> gidx;    // [G][Np] gather list: S0 without the cell, then extras
  std::vector<uint8_t> secpos;  // [(d+1)*d][Np] positions in the gather list
  std::vector<uint8_t> mask;    // [Np] bit s set = sector s alive
  std::vector<double> sigma;    // [(nb-1)*(nb-1)] oscillation matrix without row/col 0
  int64_t n_dropped = 0;
};

// Per-block halos: for each block of B consecutive cells, the sorted unique
// cells its gather lists reference (its own cells included), and every gather
// index re-expressed as a 16-bit position in that list.
struct Halo {
  int B = 0;
  int max_len = 0;                 // largest halo of any block
  std::vector<int32_t> cells;      // concatenated halos
  std::vector<int32_t> offset;     // [n_blocks + 1]
  std::vector<uint16_t> lidx;      // [G+1][Np] position of gidx[k][i] in i's block halo; row G: cell i itself
};
void build_halo(const Operators& op, int B, Halo& h);

double min_image(double delta, double L);
void build_geometry(const MeshInput& in, Geometry& g);
void face_adjacency(const MeshInput& in, std::vector<int32_t>& nbr);
void build_stencils(const Geometry& g, const std::vector<int32_t>& nbr, int n_e, int rule,
                    Stencils& st);

// Orthonormal Dubiner basis on the reference simplex.
void basis_eval(int d, int M, const double* xi, double* out);
void sigma_matrix(int d, int M, std::vector<double>& S);   // [nb][nb]
// Grundmann-Moller rule exact to `degree`: barycentric points [q][d+1], weights sum 1.
void grundmann_moller(int d, int degree, std::vector<double>& lam, std::vector<double>& w);

// Classical unstructured WENO (the scheme the paper compares CWENO with):
// 1 + 2(d+1) stencils of n_e cells each -- the central stencil, the forward
// cone sectors and the reverse cone sectors -- each with its own degree-M
// least-squares polynomial.
struct WenoStencils {
  int n_s = 0, n_e = 0;
  std::vector<int32_t> cells;    // [nc][n_s][n_e], the cell first; a row of -1 = unfillable
};
void build_weno_stencils(const Geometry& g, const std::vector<int32_t>& nbr, const Stencils& st,
                         WenoStencils& ws);

// Device layout of the WENO operators (structure of arrays, row stride Np):
//   pinv[((j * (n_e-1) + k) * (nb-1) + l) * Np + i]   stencil j, cell k+1, coefficient l+1
//   gidx[(j * (n_e-1) + k) * Np + i]                   stencil cell k+1 (the cell itself if j is dropped)
//   alive[i]                                          bit j: stencil j kept
struct WenoOperators {
  int n_s = 0;
  int64_t Np = 0, n_dropped = 0;
  std::vector<double> pinv;
  std::vector<int32_t> gidx;
  std::vector<uint16_t> alive;
};
void build_weno_operators(const Geometry& g, const WenoStencils& ws, int M, WenoOperators& op);

// Integer part of the operators: gather lists (the central stencil without
// the cell, then sector cells outside it, padded with the cell), their length
// G, the sector positions in them, and the universal Sigma.
void build_gather(const Geometry& g, const Stencils& st, int M, Operators& op);
void build_operators(const Geometry& g, const Stencils& st, int M, Operators& op);

}  // namespace cweno
