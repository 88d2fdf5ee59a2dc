// Reconstruction kernels for one (precision, dimension, degree), selected at
// compile time by CWENO_TN (f64 | f32), CWENO_D and CWENO_M; the build compiles
// this file once per combination.  Every allowed (variable block, variant)
// pair is instantiated.
#include "dispatch.hpp"

#if !defined(CWENO_TN) || !defined(CWENO_D) || !defined(CWENO_M)
#error "compile with -DCWENO_TN=f64|f32 -DCWENO_D=2|3 -DCWENO_M=1..4"
#endif

#define CWENO_CAT4(a, b, c, d) a##b##c##d
#define CWENO_NAME(tn, d, m) CWENO_CAT4(launch_, tn, _d##d, _m##m)
#define CWENO_FN(tn, d, m) CWENO_NAME(tn, d, m)
#define CWENO_BATCH_NAME(tn, d, m) CWENO_CAT4(launch_batch_, tn, _d##d, _m##m)
#define CWENO_BATCH_FN(tn, d, m) CWENO_BATCH_NAME(tn, d, m)
#define CWENO_CONF_NAME(tn, d, m) CWENO_CAT4(configure_, tn, _d##d, _m##m)
#define CWENO_PTS_NAME(tn, d, m) CWENO_CAT4(launch_points_, tn, _d##d, _m##m)
#define CWENO_PTS_FN(tn, d, m) CWENO_PTS_NAME(tn, d, m)
#define CWENO_CONF_FN(tn, d, m) CWENO_CONF_NAME(tn, d, m)
#define f64 1
#define f32 2
#if CWENO_TN == 1
typedef double real_t;
#else
typedef float real_t;
#endif
#undef f64
#undef f32

namespace cweno {
namespace {

// Fused point values: the halo kernel with chunk 1 and halo unroll 4.
template <int VB>
hipError_t launch_points_t(const KParams<real_t>& p, hipStream_t s) {
  if constexpr (vb_one_pass(CWENO_D, CWENO_M, VB, sizeof(real_t) == 4)) {
    const int64_t blocks = (p.nc + kHaloBlock - 1) / kHaloBlock;
    // block halo and a column of nb-1 blended coefficients per thread
    constexpr int NB = nbasis_c(CWENO_M, CWENO_D);
    const size_t lds = ((size_t)p.maxH * VB + (size_t)(NB - 1) * kHaloBlock) * sizeof(real_t);
    if (p.maxH <= 0 || lds > (size_t)kMaxLds || !p.phi || !p.pv || p.npts < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((reconstruct_halo_kernel<CWENO_D, CWENO_M, VB, 1, 4, real_t, true>), dim3((unsigned)blocks),
                       dim3(kHaloBlock), lds, s, p, CWENO_ARRAY_ARGS(p));
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int VB, int KC>
hipError_t launch_direct(const KParams<real_t>& p, hipStream_t s) {
  if constexpr (vb_one_pass(CWENO_D, CWENO_M, VB, sizeof(real_t) == 4)) {
    const int64_t blocks = (p.nc + kThreads - 1) / kThreads;
    hipLaunchKernelGGL((reconstruct_kernel<CWENO_D, CWENO_M, VB, KC, real_t>), dim3((unsigned)blocks),
                       dim3(kThreads), 0, s, p, CWENO_ARRAY_ARGS(p));
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

// The halo kernels' dynamic LDS limit is raised once per device by
// configure_*() (never during a launch, so that launches can be captured).
template <int VB, int KC, int HU>
hipError_t launch_halo(const KParams<real_t>& p, hipStream_t s) {
  if constexpr (vb_allowed(CWENO_D, CWENO_M, VB, sizeof(real_t) == 4)) {
    const int64_t blocks = (p.nc + kHaloBlock - 1) / kHaloBlock;
    const size_t lds = (size_t)p.maxH * VB * sizeof(real_t);
    if (p.maxH <= 0 || lds > (size_t)kMaxLds) return hipErrorInvalidValue;
    hipLaunchKernelGGL((reconstruct_halo_kernel<CWENO_D, CWENO_M, VB, KC, HU, real_t>), dim3((unsigned)blocks),
                       dim3(kHaloBlock), lds, s, p, CWENO_ARRAY_ARGS(p));
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int VB, int KC, int HU>
hipError_t launch_batch_t(const KParams<real_t>* table, const BatchItem* items, int n, int grid, size_t lds,
                          hipStream_t s) {
  if constexpr (vb_allowed(CWENO_D, CWENO_M, VB, sizeof(real_t) == 4)) {
    if (grid < 1 || n < 1 || lds == 0 || lds > (size_t)kMaxLds) return hipErrorInvalidValue;
    hipLaunchKernelGGL((reconstruct_batch_kernel<CWENO_D, CWENO_M, VB, KC, HU, real_t>), dim3((unsigned)grid),
                       dim3(kHaloBlock), lds, s, table, items, n);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int VB, int KC, int HU>
hipError_t configure_t() {
  if constexpr (vb_allowed(CWENO_D, CWENO_M, VB, sizeof(real_t) == 4)) {
    hipError_t e = hipFuncSetAttribute((const void*)reconstruct_halo_kernel<CWENO_D, CWENO_M, VB, KC, HU, real_t>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)reconstruct_batch_kernel<CWENO_D, CWENO_M, VB, KC, HU, real_t>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    if constexpr (KC == 1 && HU == 4 && vb_one_pass(CWENO_D, CWENO_M, VB, sizeof(real_t) == 4))
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)reconstruct_halo_kernel<CWENO_D, CWENO_M, VB, 1, 4, real_t, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    return e;
  } else {
    return hipSuccess;
  }
}

template <int VB>
hipError_t launch_batch_variant(const KParams<real_t>* table, const BatchItem* items, int n, int grid, size_t lds,
                                int k, hipStream_t s) {
  switch (k) {
    case 2: return launch_batch_t<VB, 1, 4>(table, items, n, grid, lds, s);
    case 3: return launch_batch_t<VB, 2, 4>(table, items, n, grid, lds, s);
    case 4: return launch_batch_t<VB, 2, 2>(table, items, n, grid, lds, s);
    case 5: return launch_batch_t<VB, 2, 8>(table, items, n, grid, lds, s);
    case 6: return launch_batch_t<VB, 4, 4>(table, items, n, grid, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int VB>
hipError_t configure_vb() {
  hipError_t e = configure_t<VB, 1, 4>();
  if (e == hipSuccess) e = configure_t<VB, 2, 4>();
  if (e == hipSuccess) e = configure_t<VB, 2, 2>();
  if (e == hipSuccess) e = configure_t<VB, 2, 8>();
  if (e == hipSuccess) e = configure_t<VB, 4, 4>();
  return e;
}

template <int VB>
hipError_t launch_variant(const KParams<real_t>& p, int k, hipStream_t s) {
  switch (k) {
    case 0: return launch_direct<VB, 1>(p, s);
    case 1: return launch_direct<VB, 2>(p, s);
    case 2: return launch_halo<VB, 1, 4>(p, s);
    case 3: return launch_halo<VB, 2, 4>(p, s);
    case 4: return launch_halo<VB, 2, 2>(p, s);
    case 5: return launch_halo<VB, 2, 8>(p, s);
    case 6: return launch_halo<VB, 4, 4>(p, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t CWENO_FN(CWENO_TN, CWENO_D, CWENO_M)(const KParams<real_t>& p, int vb, int k, hipStream_t s) {
  switch (vb) {
    case 1: return launch_variant<1>(p, k, s);
    case 2: return launch_variant<2>(p, k, s);
    case 3: return launch_variant<3>(p, k, s);
    case 4: return launch_variant<4>(p, k, s);
    case 5: return launch_variant<5>(p, k, s);
    case 9: return launch_variant<9>(p, k, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t CWENO_PTS_FN(CWENO_TN, CWENO_D, CWENO_M)(const KParams<real_t>& p, int vb, hipStream_t s) {
  switch (vb) {
    case 1: return launch_points_t<1>(p, s);
    case 2: return launch_points_t<2>(p, s);
    case 3: return launch_points_t<3>(p, s);
    case 4: return launch_points_t<4>(p, s);
    case 5: return launch_points_t<5>(p, s);
    case 9: return launch_points_t<9>(p, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t CWENO_BATCH_FN(CWENO_TN, CWENO_D, CWENO_M)(const KParams<real_t>* table, const BatchItem* items, int n,
                                                      int grid, size_t lds, int vb, int k, hipStream_t s) {
  switch (vb) {
    case 1: return launch_batch_variant<1>(table, items, n, grid, lds, k, s);
    case 2: return launch_batch_variant<2>(table, items, n, grid, lds, k, s);
    case 3: return launch_batch_variant<3>(table, items, n, grid, lds, k, s);
    case 4: return launch_batch_variant<4>(table, items, n, grid, lds, k, s);
    case 5: return launch_batch_variant<5>(table, items, n, grid, lds, k, s);
    case 9: return launch_batch_variant<9>(table, items, n, grid, lds, k, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t CWENO_CONF_FN(CWENO_TN, CWENO_D, CWENO_M)() {
  hipError_t e = configure_vb<1>();
  if (e == hipSuccess) e = configure_vb<2>();
  if (e == hipSuccess) e = configure_vb<3>();
  if (e == hipSuccess) e = configure_vb<4>();
  if (e == hipSuccess) e = configure_vb<5>();
  if (e == hipSuccess) e = configure_vb<9>();
  return e;
}

}  // namespace cweno
