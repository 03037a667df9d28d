// Binary32 instantiation of the forward kernels.
#include "mpm_kernels.hpp"

namespace mpm {
const Ops ops_f32_2d = Solver<float, 2>::table();
const Ops ops_f32_3d = Solver<float, 3>::table();
}  // namespace mpm
