// Reconstruction kernels, float precision, 2-D meshes.
#include "kernels_inst.hpp"

namespace cweno {
hipError_t launch_f32_d2(int M, int VB, const KParams<float>& p, hipStream_t s) {
  return launch_m<2, float>(M, VB, p, s);
}
}  // namespace cweno
