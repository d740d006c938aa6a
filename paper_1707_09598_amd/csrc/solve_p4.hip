// solve_p4.hip -- k_solve for spline degree 4: each inner precision, 2D (the 3D kernels are built in solve3_p4.hip).
#include "solve.hpp"

namespace igasg {

const void* solve3_kernel_p4(int prec);

const void* solve_kernel_p4(int prec, int dim) {
    if (dim == 3) return solve3_kernel_p4(prec);  // 256-thread build (solve3_p4.hip)
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<4, 0, 2>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<4, 1, 2>);
        default: return reinterpret_cast<const void*>(k_solve<4, 2, 2>);
    }
}

}  // namespace igasg
