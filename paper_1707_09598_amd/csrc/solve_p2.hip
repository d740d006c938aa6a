// solve_p2.hip -- k_solve for spline degree 2 in each inner precision.
#include "solve.hpp"

namespace igasg {

const void* solve_kernel_p2(int prec) {
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<2, 0>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<2, 1>);
        default: return reinterpret_cast<const void*>(k_solve<2, 2>);
    }
}

}  // namespace igasg
