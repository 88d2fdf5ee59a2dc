// Reconstruction kernels, double precision, 3-D meshes.
#include "kernels_inst.hpp"

namespace cweno {
hipError_t launch_f64_d3(int M, int VB, const KParams<double>& p, hipStream_t s) {
  return launch_m<3, double>(M, VB, p, s);
}
}  // namespace cweno
