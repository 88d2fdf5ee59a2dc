// Launchers of the moving-mesh kernel: one translation unit per (precision,
// dimension, degree) instantiates the segment shapes that fit that basis.
#pragma once

#include <hip/hip_runtime.h>

#include "moving_kernel.hpp"

namespace cweno {

// Segment shapes (lanes per cell, rows per lane) instantiated for (D, M): the
// rows of R must lie in the segment's row slots (fewer basis functions than
// lanes times rows per lane), three rows per lane only on 8 lanes, four only
// on 8 or 16, two rows per lane on 64 lanes only for the wide 3-D stencils,
// 4 lanes of five rows each only for the 2-D degree-3 stencils (19 cells
// besides the cell: 20 row slots against 24 on 8 lanes of three), and 8 lanes
// of eight rows each only for the 3-D degree-3 stencils (59 cells: half the
// exchange stages per sum of 16 lanes of four, at the cost of a few spilled
// registers and one workgroup per CU).
__host__ __device__ constexpr bool move_shape_ok(int D, int M, int seg, int rpl) {
  return ((seg == 4 && rpl == 5 && D == 2 && M == 3) || (seg == 8 && rpl == 8 && D == 3 && M == 3) ||
          ((seg == 8 || seg == 16 || seg == 32 || seg == 64) && rpl >= 1 && rpl <= 4)) &&
         nbasis_c(M, D) - 1 < seg * rpl && (rpl != 3 || seg == 8) && (rpl < 4 || seg <= 16) &&
         (seg < 64 || rpl == 1 || (D == 3 && M >= 2));
}

// Preferred shapes, in order: the narrowest segment whose rows hold the
// stencil, with as few rows per lane as that allows (fewer exchange stages per
// sum, more cells per wave instruction).
constexpr int kMoveShapes[13][2] = {{4, 5},  {8, 1},  {8, 2},  {8, 3},  {8, 4},  {8, 8},  {16, 1},
                                    {16, 2}, {16, 4}, {32, 1}, {32, 2}, {64, 1}, {64, 2}};

// First instantiated shape whose rows hold the NE1 stencil cells besides the
// cell (with one_row, among the shapes of one row per lane); false if none
// does.
inline bool move_shape(int D, int M, int NE1, int& seg, int& rpl, bool one_row = false) {
  for (const auto& c : kMoveShapes)
    if (move_shape_ok(D, M, c[0], c[1]) && NE1 <= c[0] * c[1] && (!one_row || c[1] == 1)) {
      seg = c[0];
      rpl = c[1];
      return true;
    }
  return false;
}

#define CWENO_DECL_MOVE(tn, T, d, m) \
  hipError_t launch_moving_##tn##_d##d##_m##m(const MParams<T>& p, int seg, int rpl, hipStream_t s);
#define CWENO_DECL_MOVE_ALL(tn, T)                                                                          \
  CWENO_DECL_MOVE(tn, T, 2, 1) CWENO_DECL_MOVE(tn, T, 2, 2) CWENO_DECL_MOVE(tn, T, 2, 3)                    \
  CWENO_DECL_MOVE(tn, T, 2, 4) CWENO_DECL_MOVE(tn, T, 3, 1) CWENO_DECL_MOVE(tn, T, 3, 2)                    \
  CWENO_DECL_MOVE(tn, T, 3, 3) CWENO_DECL_MOVE(tn, T, 3, 4)
CWENO_DECL_MOVE_ALL(f64, double)
CWENO_DECL_MOVE_ALL(f32, float)
#undef CWENO_DECL_MOVE_ALL
#undef CWENO_DECL_MOVE

#define CWENO_DECL_ASM(d, m) hipError_t launch_assemble_d##d##_m##m(const MParams<double>& p, int seg, hipStream_t s);
CWENO_DECL_ASM(2, 1) CWENO_DECL_ASM(2, 2) CWENO_DECL_ASM(2, 3) CWENO_DECL_ASM(2, 4)
CWENO_DECL_ASM(3, 1) CWENO_DECL_ASM(3, 2) CWENO_DECL_ASM(3, 3) CWENO_DECL_ASM(3, 4)
#undef CWENO_DECL_ASM

// Operator assembly on the device: p's V, C, S0, SS and SP describe the mesh,
// its pinv/binv/mask pointers receive the operators (one row per lane, so the
// central stencil may hold at most 65 cells).
inline hipError_t launch_assemble(int d, int m, const MParams<double>& p, int seg, hipStream_t s) {
  switch (d * 10 + m) {
    case 21: return launch_assemble_d2_m1(p, seg, s);
    case 22: return launch_assemble_d2_m2(p, seg, s);
    case 23: return launch_assemble_d2_m3(p, seg, s);
    case 24: return launch_assemble_d2_m4(p, seg, s);
    case 31: return launch_assemble_d3_m1(p, seg, s);
    case 32: return launch_assemble_d3_m2(p, seg, s);
    case 33: return launch_assemble_d3_m3(p, seg, s);
    case 34: return launch_assemble_d3_m4(p, seg, s);
  }
  return hipErrorInvalidValue;
}

#define CWENO_MOVE_CASES(tn)                                                             \
  switch (d * 10 + m) {                                                                  \
    case 21: return launch_moving_##tn##_d2_m1(p, seg, rpl, s);                          \
    case 22: return launch_moving_##tn##_d2_m2(p, seg, rpl, s);                          \
    case 23: return launch_moving_##tn##_d2_m3(p, seg, rpl, s);                          \
    case 24: return launch_moving_##tn##_d2_m4(p, seg, rpl, s);                          \
    case 31: return launch_moving_##tn##_d3_m1(p, seg, rpl, s);                          \
    case 32: return launch_moving_##tn##_d3_m2(p, seg, rpl, s);                          \
    case 33: return launch_moving_##tn##_d3_m3(p, seg, rpl, s);                          \
    case 34: return launch_moving_##tn##_d3_m4(p, seg, rpl, s);                          \
  }                                                                                      \
  return hipErrorInvalidValue;

inline hipError_t launch_moving(int d, int m, const MParams<double>& p, int seg, int rpl, hipStream_t s) {
  CWENO_MOVE_CASES(f64)
}
inline hipError_t launch_moving(int d, int m, const MParams<float>& p, int seg, int rpl, hipStream_t s) {
  CWENO_MOVE_CASES(f32)
}
#undef CWENO_MOVE_CASES

}  // namespace cweno
