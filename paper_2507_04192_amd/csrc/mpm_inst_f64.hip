// Binary64 instantiation of the forward kernels.
#include "mpm_kernels.hpp"

namespace mpm {
const Ops ops_f64_2d = Solver<double, 2>::table();
const Ops ops_f64_3d = Solver<double, 3>::table();
}  // namespace mpm
