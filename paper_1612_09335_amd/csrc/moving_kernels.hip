// Moving-mesh kernels for one (precision, dimension, degree), selected at
// compile time by CWENO_TN (f64 | f32), CWENO_D and CWENO_M; the build compiles
// this file once per combination.
#include "moving.hpp"

#if !defined(CWENO_TN) || !defined(CWENO_D) || !defined(CWENO_M)
#error "compile with -DCWENO_TN=f64|f32 -DCWENO_D=2|3 -DCWENO_M=1..4"
#endif

#define CWENO_CAT4(a, b, c, d) a##b##c##d
#define CWENO_MOVE_NAME(tn, d, m) CWENO_CAT4(launch_moving_, tn, _d##d, _m##m)
#define CWENO_MOVE_FN(tn, d, m) CWENO_MOVE_NAME(tn, d, m)
#define CWENO_ASM_NAME(d, m) CWENO_CAT4(launch_assemble, _d, d, _m##m)
#define CWENO_ASM_FN(d, m) CWENO_ASM_NAME(d, m)
#define f64 1
#define f32 2
#if CWENO_TN == 1
typedef double real_t;
#define CWENO_TN_IS_F64 1
#else
typedef float real_t;
#define CWENO_TN_IS_F64 0
#endif
#undef f64
#undef f32

namespace cweno {
namespace {

template <int SEG, int RPL, int VB>
hipError_t launch_vb(const MParams<real_t>& p, hipStream_t s) {
  // only the pass sizes this shape uses (move_vb of VB variables is VB)
  if constexpr (VB <= move_vb_max(CWENO_D, CWENO_M, SEG) && move_vb(CWENO_D, CWENO_M, SEG, VB) == VB) {
    constexpr int cpb = (kMoveThreads / 64) * (64 / SEG);
    const int64_t blocks = (p.nc + cpb - 1) / cpb;
    hipLaunchKernelGGL((moving_kernel<CWENO_D, CWENO_M, SEG, RPL, VB, real_t>), dim3((unsigned)blocks),
                       dim3(kMoveThreads), 0, s, p);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int SEG, int RPL>
hipError_t launch_shape(const MParams<real_t>& p, hipStream_t s) {
  if constexpr (move_shape_ok(CWENO_D, CWENO_M, SEG, RPL)) {
    switch (move_vb(CWENO_D, CWENO_M, SEG, p.nv)) {
      case 2: return launch_vb<SEG, RPL, 2>(p, s);
      case 4: return launch_vb<SEG, RPL, 4>(p, s);
      case 5: return launch_vb<SEG, RPL, 5>(p, s);
      case 9: return launch_vb<SEG, RPL, 9>(p, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

#if CWENO_TN_IS_F64
// Operator assembly (one row per lane) for this (dimension, degree).
hipError_t CWENO_ASM_FN(CWENO_D, CWENO_M)(const MParams<double>& p, int seg, hipStream_t s) {
  auto go = [&](auto segc) -> hipError_t {
    constexpr int SEG = decltype(segc)::value;
    if constexpr (move_shape_ok(CWENO_D, CWENO_M, SEG, 1)) {
      constexpr int cpb = (kMoveThreads / 64) * (64 / SEG);
      const int64_t blocks = (p.nc + cpb - 1) / cpb;
      hipLaunchKernelGGL((moving_kernel<CWENO_D, CWENO_M, SEG, 1, 0, double>), dim3((unsigned)blocks),
                         dim3(kMoveThreads), 0, s, p);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  };
  if (seg == 8) return go(std::integral_constant<int, 8>{});
  if (seg == 16) return go(std::integral_constant<int, 16>{});
  if (seg == 32) return go(std::integral_constant<int, 32>{});
  if (seg == 64) return go(std::integral_constant<int, 64>{});
  return hipErrorInvalidValue;
}
#endif

hipError_t CWENO_MOVE_FN(CWENO_TN, CWENO_D, CWENO_M)(const MParams<real_t>& p, int seg, int rpl, hipStream_t s) {
  if (seg == 4 && rpl == 5) return launch_shape<4, 5>(p, s);
  if (seg == 8 && rpl == 8) return launch_shape<8, 8>(p, s);
  if (seg == 8 && rpl == 1) return launch_shape<8, 1>(p, s);
  if (seg == 8 && rpl == 2) return launch_shape<8, 2>(p, s);
  if (seg == 8 && rpl == 3) return launch_shape<8, 3>(p, s);
  if (seg == 8 && rpl == 4) return launch_shape<8, 4>(p, s);
  if (seg == 16 && rpl == 1) return launch_shape<16, 1>(p, s);
  if (seg == 16 && rpl == 2) return launch_shape<16, 2>(p, s);
  if (seg == 16 && rpl == 4) return launch_shape<16, 4>(p, s);
  if (seg == 32 && rpl == 1) return launch_shape<32, 1>(p, s);
  if (seg == 32 && rpl == 2) return launch_shape<32, 2>(p, s);
  if (seg == 64 && rpl == 1) return launch_shape<64, 1>(p, s);
  if (seg == 64 && rpl == 2) return launch_shape<64, 2>(p, s);
  return hipErrorInvalidValue;
}

}  // namespace cweno
