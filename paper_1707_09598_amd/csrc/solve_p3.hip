// solve_p3.hip -- k_solve for spline degree 3: each inner precision, 2D (the 3D kernels are built in solve3_p3.hip).
#include "solve.hpp"

namespace igasg {

const void* solve3_kernel_p3(int prec);

const void* solve_kernel_p3(int prec, int dim) {
    if (dim == 3) return solve3_kernel_p3(prec);  // 256-thread build (solve3_p3.hip)
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<3, 0, 2>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<3, 1, 2>);
        default: return reinterpret_cast<const void*>(k_solve<3, 2, 2>);
    }
}

}  // namespace igasg
