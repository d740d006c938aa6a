// solve3_p1.hip -- k_solve for spline degree 1 in 3D, each inner precision,
// built with 256-thread workgroups (see IGASG_THREADS in common.hpp).
#define IGASG_THREADS 256
#include "solve.hpp"

namespace igasg {

const void* solve3_kernel_p1(int prec, int grid) {
    if (grid) {
        switch (prec) {
            case IGA_PREC_FP64: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 0, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 0, 3, kBlock, 1>);
            case IGA_PREC_FP32: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 1, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 1, 3, kBlock, 1>);
            default: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 2, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 2, 3, kBlock, 1>);
        }
    }
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<1, 0, 3, kBlock>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<1, 1, 3, kBlock>);
        default: return reinterpret_cast<const void*>(k_solve<1, 2, 3, kBlock>);
    }
}

}  // namespace igasg
