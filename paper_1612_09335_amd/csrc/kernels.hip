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

template <int VB, int RS, int KC>
hipError_t launch_one(const KParams<real_t>& p, hipStream_t s) {
  if constexpr (vb_allowed(CWENO_D, CWENO_M, VB, RS, sizeof(real_t) == 4)) {
    constexpr int cpb = kThreads / RS;
    const int64_t blocks = (p.nc + cpb - 1) / cpb;
    constexpr int lds = lds_bytes<CWENO_D, CWENO_M, VB, RS, real_t>();
    hipLaunchKernelGGL((reconstruct_kernel<CWENO_D, CWENO_M, VB, RS, KC, real_t>), dim3((unsigned)blocks),
                       dim3(kThreads), lds, s, p);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int VB>
hipError_t launch_variant(const KParams<real_t>& p, int rs, int kc, hipStream_t s) {
  if (rs == 1 && kc == 1) return launch_one<VB, 1, 1>(p, s);
  if (rs == 1 && kc == 2) return launch_one<VB, 1, 2>(p, s);
  if (rs == 2 && kc == 2) return launch_one<VB, 2, 2>(p, s);
  if (rs == 2 && kc == 4) return launch_one<VB, 2, 4>(p, s);
  if (rs == 4 && kc == 2) return launch_one<VB, 4, 2>(p, s);
  if (rs == 4 && kc == 4) return launch_one<VB, 4, 4>(p, s);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t CWENO_FN(CWENO_TN, CWENO_D, CWENO_M)(const KParams<real_t>& p, int vb, int rs, int kc, hipStream_t s) {
  switch (vb) {
    case 1: return launch_variant<1>(p, rs, kc, s);
    case 2: return launch_variant<2>(p, rs, kc, s);
    case 3: return launch_variant<3>(p, rs, kc, s);
    case 4: return launch_variant<4>(p, rs, kc, s);
    case 5: return launch_variant<5>(p, rs, kc, s);
    case 9: return launch_variant<9>(p, rs, kc, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cweno
