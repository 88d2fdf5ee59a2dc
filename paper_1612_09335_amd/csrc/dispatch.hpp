// Host-side dispatch of the templated reconstruction kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "reconstruct_kernel.hpp"

namespace cweno {

// Variable-block sizes that are instantiated.  A block of VB variables keeps
// (n_basis-1)*VB accumulators per thread; blocks whose accumulators would not
// fit the register budget (100 doubles / 200 floats) are not instantiated.
__host__ __device__ constexpr bool vb_allowed(int D, int M, int VB, bool f32) {
  return (VB == 1 || VB == 2 || VB == 3 || VB == 4 || VB == 5 || VB == 9) &&
         (nbasis_c(M, D) - 1) * VB <= (f32 ? 200 : 100);
}

// Largest instantiated block size not above n.
inline int pick_vb(int D, int M, int n, bool f32) {
  const int cand[] = {9, 5, 4, 3, 2, 1};
  for (int vb : cand)
    if (vb <= n && vb_allowed(D, M, vb, f32)) return vb;
  return 1;
}

hipError_t launch_f64_d2(int M, int VB, const KParams<double>& p, hipStream_t s);
hipError_t launch_f64_d3(int M, int VB, const KParams<double>& p, hipStream_t s);
hipError_t launch_f32_d2(int M, int VB, const KParams<float>& p, hipStream_t s);
hipError_t launch_f32_d3(int M, int VB, const KParams<float>& p, hipStream_t s);

}  // namespace cweno
