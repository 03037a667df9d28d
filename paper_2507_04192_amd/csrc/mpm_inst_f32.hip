// Binary32 instantiation of the forward kernels.
#include "mpm_adjoint.hpp"

namespace mpm {
template <class T, int D>
static Ops with_adjoint()
{
    Ops o = Solver<T, D>::table();
    o.forward_loss = &Adjoint<T, D>::forward_loss;
    o.backward = &Adjoint<T, D>::backward;
    o.extract = &Adjoint<T, D>::extract;
    return o;
}

const Ops ops_f32_2d = with_adjoint<float, 2>();
const Ops ops_f32_3d = with_adjoint<float, 3>();
}  // namespace mpm
