// solve_p1.hip -- k_solve for spline degree 1: each inner precision, 2D and 3D.
#include "solve.hpp"

namespace igasg {

const void* solve_kernel_p1(int prec, int dim) {
    if (dim == 3) {
        switch (prec) {
            case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<1, 0, 3>);
            case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<1, 1, 3>);
            default: return reinterpret_cast<const void*>(k_solve<1, 2, 3>);
        }
    }
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<1, 0, 2>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<1, 1, 2>);
        default: return reinterpret_cast<const void*>(k_solve<1, 2, 2>);
    }
}

}  // namespace igasg
