// solve_p4.hip -- k_solve for spline degree 4 in each inner precision.
#include "solve.hpp"

namespace igasg {

const void* solve_kernel_p4(int prec) {
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<4, 0>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<4, 1>);
        default: return reinterpret_cast<const void*>(k_solve<4, 2>);
    }
}

}  // namespace igasg
