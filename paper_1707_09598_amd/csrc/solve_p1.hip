// solve_p1.hip -- k_solve for spline degree 1 in each inner precision.
#include "solve.hpp"

namespace igasg {

const void* solve_kernel_p1(int prec) {
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<1, 0>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<1, 1>);
        default: return reinterpret_cast<const void*>(k_solve<1, 2>);
    }
}

}  // namespace igasg
