// Reconstruction kernels, double precision, 2-D meshes.
#include "kernels_inst.hpp"

namespace cweno {
hipError_t launch_f64_d2(int M, int VB, const KParams<double>& p, hipStream_t s) {
  return launch_m<2, double>(M, VB, p, s);
}
}  // namespace cweno
