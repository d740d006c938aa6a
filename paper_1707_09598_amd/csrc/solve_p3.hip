// solve_p3.hip -- k_solve for spline degree 3 in each inner precision.
#include "solve.hpp"

namespace igasg {

const void* solve_kernel_p3(int prec) {
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<3, 0>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<3, 1>);
        default: return reinterpret_cast<const void*>(k_solve<3, 2>);
    }
}

}  // namespace igasg
