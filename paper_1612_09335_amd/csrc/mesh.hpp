// Library-internal view of a registered mesh (shared by the C ABI's
// translation units; not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cweno.h"
#include "dispatch.hpp"
#include "host.hpp"

namespace cweno_abi {

// Records the detail string returned by cweno_last_error (thread-local).
cweno_status fail(cweno_status st, const std::string& msg);

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Whether [a, a + na) and [b, b + nb) share a byte (empty ranges never do).
inline bool overlap(const void* a, uint64_t na, const void* b, uint64_t nb) {
  if (!a || !b || !na || !nb) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// For every sector cell of every cell, its row in the central stencil (its
// position there minus one) or 255 if it is not in it: [nc][d+1][d]
// (the moving-mesh kernel reads such cells' barycentres from its row lanes).
inline std::vector<uint8_t> sector_rows(int d, int64_t nc, int n_e, const std::vector<int32_t>& central,
                                        const std::vector<int32_t>& sectors) {
  const int ns = d + 1;
  std::vector<uint8_t> out((size_t)nc * ns * d, 255);
  for (int64_t i = 0; i < nc; ++i) {
    const int32_t* S0 = &central[(size_t)i * n_e];
    for (int s = 0; s < ns; ++s) {
      const int32_t* sec = &sectors[((size_t)i * ns + s) * ns];
      if (sec[0] < 0) continue;
      for (int a = 0; a < d; ++a)
        for (int k = 1; k < n_e && k <= 255; ++k)
          if (S0[k] == sec[a + 1]) {
            out[((size_t)i * ns + s) * d + a] = (uint8_t)(k - 1);
            break;
          }
    }
  }
  return out;
}

// Raise the dynamic-LDS limit of every halo kernel once per device (before
// any launch, so that launches may later be captured into graphs).
cweno_status configure_device_kernels();

}  // namespace cweno_abi

struct cweno_mesh {
  int d = 2, M = 1, nb = 0, n_e = 0, G = 0;
  int64_t nc = 0, Np = 0;
  double lam[5] = {0, 0, 0, 0, 0};
  double eps = 1e-14;
  int r = 4;
  unsigned flags = 0;
  int ops = CWENO_OPS_F64;
  int64_t n_dropped = 0;
  // host copies
  std::vector<int32_t> nbr, central, sectors;
  cweno::Operators op;  // FP64 operators (host copy kept only for host-only meshes)
  // device residency
  int device = -1;
  cweno_abi::DevBuf pinv64, binv64, sigma64, pinv32, binv32, sigma32, gidx, secpos, mask, halo, hoff, lidx;
  int maxH = 0;
  // moving meshes: cell vertex ids, central and sector stencils (cell-major),
  // each sector cell's row in the central stencil
  cweno_abi::DevBuf mvC, mvS0, mvSS, mvSP;
  int mv_seg = 0, mv_rpl = 0;   // work mapping set by the caller; 0 = the default shape
  int64_t n_vertices = 0;
  // classical WENO meshes (n_s > 0): stencil tables [nc][n_s][n_e] on the host;
  // operators, kept-stencil bits and the halos of blocks of 64 cells (cells,
  // offsets, 16-bit positions of every stencil entry) on the device
  int n_s = 0;
  std::vector<int32_t> weno_cells;
  cweno_abi::DevBuf wpinv, walive, whalo, whoff, wlidx;
  int wmaxH = 0;
  double box[3] = {0, 0, 0};
  int64_t device_bytes = 0;
  bool owns_device = true;   // false: the device buffers point into memory owned elsewhere (a server arena)
  // kernel variant (index into cweno::kVariants) per [precision][variable block]
  int variant[2][10];

  ~cweno_mesh() {
    if (!owns_device) return;
    for (cweno_abi::DevBuf* b : {&pinv64, &binv64, &sigma64, &pinv32, &binv32, &sigma32, &gidx, &secpos, &mask, &halo,
                                 &hoff, &lidx, &mvC, &mvS0, &mvSS, &mvSP, &wpinv, &walive, &whalo, &whoff, &wlidx})
      if (b->p) (void)hipFree(b->p);
  }
};

namespace cweno_abi {

// Whether variant k can run blocks of vb variables on this mesh: instantiated,
// and for the halo kernel, the block halos fit in LDS.
inline bool variant_ok(const cweno_mesh* m, int vb, int k, bool f32) {
  const cweno::Variant& V = cweno::kVariants[k];
  if (!cweno::variant_allowed(m->d, m->M, vb, V, f32)) return false;
  // the halo kernel stages a block of vb variables through one 32-bit offset range
  if (V.kind == 1)
    return m->maxH > 0 && (int64_t)m->maxH * vb * (f32 ? 4 : 8) <= cweno::kMaxLds &&
           (uint64_t)vb * (uint64_t)m->nc * (f32 ? 4u : 8u) < (uint64_t(1) << 32);
  return true;
}

// Default variant: the candidate order below, first one that can run.
inline int default_variant(const cweno_mesh* m, int vb, bool f32) {
  const int order[] = {3, 2, 4, 5, 6, 1, 0};
  for (int k : order)
    if (variant_ok(m, vb, k, f32)) return k;
  return -1;
}

// Largest variable block not above n that this mesh can run: some variant
// (with halo_only, an LDS-halo variant) is instantiated for it and, for the
// halo kernel, the mesh's block halos of that many variables fit in LDS.
inline int pick_vb_mesh(const cweno_mesh* m, int n, bool f32, bool halo_only = false) {
  const int cand[] = {9, 5, 4, 3, 2, 1};
  for (int vb : cand) {
    if (vb > n) continue;
    for (int k = 0; k < cweno::kNumVariants; ++k)
      if ((!halo_only || cweno::kVariants[k].kind == 1) && variant_ok(m, vb, k, f32)) return vb;
  }
  return 1;
}

template <typename T>
inline cweno::KParams<T> make_params(const cweno_mesh* m, const void* q, void* coeffs, void* sigma, void* omega, int v0) {
  const bool f32 = sizeof(T) == 4;
  cweno::KParams<T> p{};
  p.q = (const T*)q;
  p.out = (T*)coeffs;
  p.sig = (T*)sigma;
  p.om = (T*)omega;
  p.pinv = (const T*)(f32 ? m->pinv32.p : m->pinv64.p);
  p.binv = (const T*)(f32 ? m->binv32.p : m->binv64.p);
  p.sigma = (const T*)(f32 ? m->sigma32.p : m->sigma64.p);
  p.gidx = (const int32_t*)m->gidx.p;
  p.secpos = (const uint8_t*)m->secpos.p;
  p.mask = (const uint8_t*)m->mask.p;
  p.halo = (const int32_t*)m->halo.p;
  p.hoff = (const int32_t*)m->hoff.p;
  p.lidx = (const uint16_t*)m->lidx.p;
  p.maxH = m->maxH;
  p.G = m->G;
  p.nc = m->nc;
  p.Np = m->Np;
  p.NE1 = m->n_e - 1;
  p.v0 = v0;
  p.r = m->r;
  p.sigma0_popt = (m->flags & CWENO_FLAG_SIGMA0_POPT) ? 1 : 0;
  p.linear_w = (m->flags & CWENO_FLAG_LINEAR_WEIGHTS) ? 1 : 0;
  for (int t = 0; t < 5; ++t) p.lam[t] = (T)m->lam[t];
  p.eps = (T)m->eps;
  return p;
}

// Launch one variable block [v0, v0+vb) with variant index k.
inline hipError_t launch_block(const cweno_mesh* m, bool f32, const void* q, void* coeffs, void* sigma, void* omega,
                        int v0, int vb, int k, hipStream_t s) {
  if (f32)
    return cweno::launch<float>(m->d, m->M, make_params<float>(m, q, coeffs, sigma, omega, v0), vb, k, s);
  return cweno::launch<double>(m->d, m->M, make_params<double>(m, q, coeffs, sigma, omega, v0), vb, k, s);
}

}  // namespace cweno_abi
