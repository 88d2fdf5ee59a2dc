// Host-side dispatch of the templated reconstruction kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "reconstruct_kernel.hpp"
#include "pc_kernel.hpp"
#include "halo_kernel.hpp"

namespace cweno {

// Kernel variants.  pc == 0: reconstruct_kernel with rs lanes per cell and
// kc stencil entries per chunk.  pc == 1: reconstruct_pc_kernel with rs
// consumer wavefronts, a producer kc entries ahead and gathers p entries ahead.
// pc == 2: reconstruct_halo_kernel (stencil values from an LDS halo) with
// kc stencil entries per chunk.
struct Variant { int rs, kc, pc, p; };
constexpr Variant kVariants[] = {{1, 1, 0, 0}, {1, 2, 0, 0}, {2, 2, 0, 0}, {2, 4, 0, 0}, {4, 2, 0, 0},
                                 {4, 4, 0, 0}, {3, 3, 1, 1}, {2, 4, 1, 1}, {1, 5, 1, 1}, {1, 1, 2, 0},
                                 {1, 2, 2, 0}, {1, 4, 2, 0}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Variable-block sizes that are instantiated.  A lane keeps
// ceil((n_basis-1)/RS) * VB accumulators; combinations whose accumulators
// exceed the register budget (100 doubles / 200 floats) or whose row exchange
// exceeds the 160 KiB of LDS a workgroup may use are not instantiated.
constexpr int kMaxLds = 160 * 1024;
__host__ __device__ constexpr bool vb_allowed(int D, int M, int VB, int RS, bool f32) {
  return (VB == 1 || VB == 2 || VB == 3 || VB == 4 || VB == 5 || VB == 9) &&
         ceil_div(nbasis_c(M, D) - 1, RS) * VB <= (f32 ? 200 : 100) &&
         (RS == 1 ? 0 : (kThreads / RS) * (nbasis_c(M, D) - 1) * VB * (f32 ? 4 : 8)) <= kMaxLds;
}

// Producer/consumer kernel: consumer accumulators as above, the producer's
// register ring (DP entries of 16-byte chunks) within 240 VGPRs, two stages in LDS.
__host__ __device__ constexpr bool pc_allowed(int D, int M, int VB, int NCW, int DP, bool f32) {
  return vb_allowed(D, M, VB, 1, f32) &&
         DP * 4 * (((nbasis_c(M, D) - 1) * 64 * NCW * (f32 ? 4 : 8) / 16 + 16 * NCW + 63) / 64) <= 240 &&
         2 * ((nbasis_c(M, D) - 1) * 64 * NCW * (f32 ? 4 : 8) + 256 * NCW) <= kMaxLds;
}

__host__ __device__ constexpr bool variant_allowed(int D, int M, int VB, const Variant& v, bool f32) {
  return v.pc == 0   ? vb_allowed(D, M, VB, v.rs, f32)
         : v.pc == 1 ? pc_allowed(D, M, VB, v.rs, v.kc, f32)
                     : vb_allowed(D, M, VB, 1, f32);
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

#define CWENO_DECLARE(TN, T, D, M) \
  hipError_t launch_##TN##_d##D##_m##M(const KParams<T>& p, int vb, int k, hipStream_t s);
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

}  // namespace cweno
