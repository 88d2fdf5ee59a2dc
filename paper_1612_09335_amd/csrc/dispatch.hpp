// Host-side dispatch of the templated reconstruction kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "reconstruct_kernel.hpp"
#include "halo_kernel.hpp"

namespace cweno {

// Kernel variants.  kind 0: reconstruct_kernel (neighbour averages gathered
// from global memory), kc stencil entries per chunk.  kind 1:
// reconstruct_halo_kernel (neighbour averages from the block's LDS halo), kc
// stencil entries per chunk, halo staged hu entries per thread at a time.
struct Variant { int kind, kc, hu; };
constexpr Variant kVariants[] = {{0, 1, 0}, {0, 2, 0}, {1, 1, 4}, {1, 2, 4}, {1, 2, 2}, {1, 2, 8}, {1, 4, 4}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Variable-block sizes that are instantiated.  A lane keeps (n_basis-1) * VB
// accumulators; the direct kernel (and the fused point-value form) only
// blocks whose accumulators fit the register budget (100 doubles / 200
// floats), the LDS-halo kernel also blocks up to twice that, walking the
// stencil twice for half of P_opt's rows each time.  The halo kernel also
// needs maxH * VB values of LDS, at most the 160 KiB a workgroup may use.
constexpr int kMaxLds = 160 * 1024;
__host__ __device__ constexpr bool vb_size_ok(int VB) {
  return VB == 1 || VB == 2 || VB == 3 || VB == 4 || VB == 5 || VB == 9;
}
__host__ __device__ constexpr bool vb_one_pass(int D, int M, int VB, bool f32) {
  return vb_size_ok(VB) && (nbasis_c(M, D) - 1) * VB <= acc_budget(f32);
}
__host__ __device__ constexpr bool vb_allowed(int D, int M, int VB, bool f32) {
  return vb_size_ok(VB) && (nbasis_c(M, D) - 1) * VB <= 2 * acc_budget(f32);
}

__host__ __device__ constexpr bool variant_allowed(int D, int M, int VB, const Variant& V, bool f32) {
  return V.kind == 0 ? vb_one_pass(D, M, VB, f32) : vb_allowed(D, M, VB, f32);
}

// Largest block size not above n that some variant instantiates.
inline int pick_vb(int D, int M, int n, bool f32) {
  const int cand[] = {9, 5, 4, 3, 2, 1};
  for (int vb : cand)
    if (vb <= n)
      for (const Variant& v : kVariants)
        if (variant_allowed(D, M, vb, v, f32)) return vb;
  return 1;
}

// Largest block size not above n whose accumulators fit one pass (the fused
// point-value form walks the stencil once).
inline int pick_vb_one_pass(int D, int M, int n, bool f32) {
  const int cand[] = {9, 5, 4, 3, 2, 1};
  for (int vb : cand)
    if (vb <= n && vb_one_pass(D, M, vb, f32)) return vb;
  return 1;
}

// Per (precision, dimension, degree) unit: one-mesh launch, batched launch
// (work list over a device table of meshes), and the one-time setting of the
// dynamic-LDS limit of the unit's halo kernels (outside any stream capture).
#define CWENO_DECLARE(TN, T, D, M)                                                                    \
  hipError_t launch_##TN##_d##D##_m##M(const KParams<T>& p, int vb, int k, hipStream_t s);           \
  hipError_t launch_points_##TN##_d##D##_m##M(const KParams<T>& p, int vb, hipStream_t s);           \
  hipError_t launch_batch_##TN##_d##D##_m##M(const KParams<T>* table, const BatchItem* items, int n, \
                                             int grid, size_t lds, int vb, int k, hipStream_t s);    \
  hipError_t configure_##TN##_d##D##_m##M();
#define CWENO_DECLARE_T(TN, T) \
  CWENO_DECLARE(TN, T, 2, 1) CWENO_DECLARE(TN, T, 2, 2) CWENO_DECLARE(TN, T, 2, 3) CWENO_DECLARE(TN, T, 2, 4) \
  CWENO_DECLARE(TN, T, 3, 1) CWENO_DECLARE(TN, T, 3, 2) CWENO_DECLARE(TN, T, 3, 3) CWENO_DECLARE(TN, T, 3, 4)
CWENO_DECLARE_T(f64, double)
CWENO_DECLARE_T(f32, float)
#undef CWENO_DECLARE_T
#undef CWENO_DECLARE

template <typename T>
inline hipError_t launch(int D, int M, const KParams<T>& p, int vb, int k, hipStream_t s) {
#define CWENO_CASE(TN, DD, MM) \
  if (D == DD && M == MM) return launch_##TN##_d##DD##_m##MM(p, vb, k, s);
  if constexpr (sizeof(T) == 8) {
    CWENO_CASE(f64, 2, 1) CWENO_CASE(f64, 2, 2) CWENO_CASE(f64, 2, 3) CWENO_CASE(f64, 2, 4)
    CWENO_CASE(f64, 3, 1) CWENO_CASE(f64, 3, 2) CWENO_CASE(f64, 3, 3) CWENO_CASE(f64, 3, 4)
  } else {
    CWENO_CASE(f32, 2, 1) CWENO_CASE(f32, 2, 2) CWENO_CASE(f32, 2, 3) CWENO_CASE(f32, 2, 4)
    CWENO_CASE(f32, 3, 1) CWENO_CASE(f32, 3, 2) CWENO_CASE(f32, 3, 3) CWENO_CASE(f32, 3, 4)
  }
#undef CWENO_CASE
  return hipErrorInvalidValue;
}

template <typename T>
inline hipError_t launch_batch(int D, int M, const KParams<T>* table, const BatchItem* items, int n, int grid,
                               size_t lds, int vb, int k, hipStream_t s) {
#define CWENO_CASE(TN, DD, MM) \
  if (D == DD && M == MM) return launch_batch_##TN##_d##DD##_m##MM(table, items, n, grid, lds, vb, k, s);
  if constexpr (sizeof(T) == 8) {
    CWENO_CASE(f64, 2, 1) CWENO_CASE(f64, 2, 2) CWENO_CASE(f64, 2, 3) CWENO_CASE(f64, 2, 4)
    CWENO_CASE(f64, 3, 1) CWENO_CASE(f64, 3, 2) CWENO_CASE(f64, 3, 3) CWENO_CASE(f64, 3, 4)
  } else {
    CWENO_CASE(f32, 2, 1) CWENO_CASE(f32, 2, 2) CWENO_CASE(f32, 2, 3) CWENO_CASE(f32, 2, 4)
    CWENO_CASE(f32, 3, 1) CWENO_CASE(f32, 3, 2) CWENO_CASE(f32, 3, 3) CWENO_CASE(f32, 3, 4)
  }
#undef CWENO_CASE
  return hipErrorInvalidValue;
}

// The halo kernel (chunk 1, halo unroll 4) writing the reconstruction's values
// at a point set (p.phi, p.pv, p.npts) instead of its coefficients.
template <typename T>
inline hipError_t launch_points(int D, int M, const KParams<T>& p, int vb, hipStream_t s) {
#define CWENO_CASE(TN, DD, MM) \
  if (D == DD && M == MM) return launch_points_##TN##_d##DD##_m##MM(p, vb, s);
  if constexpr (sizeof(T) == 8) {
    CWENO_CASE(f64, 2, 1) CWENO_CASE(f64, 2, 2) CWENO_CASE(f64, 2, 3) CWENO_CASE(f64, 2, 4)
    CWENO_CASE(f64, 3, 1) CWENO_CASE(f64, 3, 2) CWENO_CASE(f64, 3, 3) CWENO_CASE(f64, 3, 4)
  } else {
    CWENO_CASE(f32, 2, 1) CWENO_CASE(f32, 2, 2) CWENO_CASE(f32, 2, 3) CWENO_CASE(f32, 2, 4)
    CWENO_CASE(f32, 3, 1) CWENO_CASE(f32, 3, 2) CWENO_CASE(f32, 3, 3) CWENO_CASE(f32, 3, 4)
  }
#undef CWENO_CASE
  return hipErrorInvalidValue;
}

// Allow every halo kernel of every unit the full LDS of a workgroup (on the
// current device).
inline hipError_t configure_all() {
  hipError_t (*const fns[])() = {
      configure_f64_d2_m1, configure_f64_d2_m2, configure_f64_d2_m3, configure_f64_d2_m4,
      configure_f64_d3_m1, configure_f64_d3_m2, configure_f64_d3_m3, configure_f64_d3_m4,
      configure_f32_d2_m1, configure_f32_d2_m2, configure_f32_d2_m3, configure_f32_d2_m4,
      configure_f32_d3_m1, configure_f32_d3_m2, configure_f32_d3_m3, configure_f32_d3_m4};
  for (auto f : fns) {
    const hipError_t e = f();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cweno
