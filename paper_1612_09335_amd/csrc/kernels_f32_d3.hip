// Reconstruction kernels, float precision, 3-D meshes.
#include "kernels_inst.hpp"

namespace cweno {
hipError_t launch_f32_d3(int M, int VB, const KParams<float>& p, hipStream_t s) {
  return launch_m<3, float>(M, VB, p, s);
}
}  // namespace cweno
