// solve3_p4.hip -- k_solve for spline degree 4 in 3D, each inner precision,
// built with 256-thread workgroups (see IGASG_THREADS in common.hpp).
#define IGASG_THREADS 256
#include "solve.hpp"

namespace igasg {

const void* solve3_kernel_p4(int prec, int grid) {
    if (grid) {
        switch (prec) {
            case IGA_PREC_FP64: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<4, 0, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<4, 0, 3, kBlock, 1>);
            case IGA_PREC_FP32: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<4, 1, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<4, 1, 3, kBlock, 1>);
            default: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<4, 2, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<4, 2, 3, kBlock, 1>);
        }
    }
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<4, 0, 3, kBlock>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<4, 1, 3, kBlock>);
        default: return reinterpret_cast<const void*>(k_solve<4, 2, 3, kBlock>);
    }
}

}  // namespace igasg
