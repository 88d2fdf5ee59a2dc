// Instantiation helper: expands the (M, VB) switch for one (T, D) pair.
#pragma once

#include "dispatch.hpp"

namespace cweno {

template <int D, int M, int VB, typename T>
hipError_t launch_one(const KParams<T>& p, hipStream_t s) {
  if constexpr (vb_allowed(D, M, VB, sizeof(T) == 4)) {
    const int64_t blocks = (p.nc + kThreads - 1) / kThreads;
    hipLaunchKernelGGL((reconstruct_kernel<D, M, VB, T>), dim3((unsigned)blocks), dim3(kThreads), 0, s, p);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int D, int M, typename T>
hipError_t launch_vb(int VB, const KParams<T>& p, hipStream_t s) {
  switch (VB) {
    case 1: return launch_one<D, M, 1, T>(p, s);
    case 2: return launch_one<D, M, 2, T>(p, s);
    case 3: return launch_one<D, M, 3, T>(p, s);
    case 4: return launch_one<D, M, 4, T>(p, s);
    case 5: return launch_one<D, M, 5, T>(p, s);
    case 9: return launch_one<D, M, 9, T>(p, s);
    default: return hipErrorInvalidValue;
  }
}

template <int D, typename T>
hipError_t launch_m(int M, int VB, const KParams<T>& p, hipStream_t s) {
  switch (M) {
    case 1: return launch_vb<D, 1, T>(VB, p, s);
    case 2: return launch_vb<D, 2, T>(VB, p, s);
    case 3: return launch_vb<D, 3, T>(VB, p, s);
    case 4: return launch_vb<D, 4, T>(VB, p, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cweno
