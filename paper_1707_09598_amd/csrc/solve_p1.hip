// solve_p1.hip -- k_solve for spline degree 1: each inner precision, 2D and 3D
// with 512-thread workgroups (the 256-thread 3D build is solve3_p1.hip).
#include "solve.hpp"

namespace igasg {

const void* solve3_kernel_p1(int prec, int grid);

const void* solve_kernel_p1(int prec, int dim, int narrow, int grid) {
    if (dim == 3 && narrow) return solve3_kernel_p1(prec, grid);  // 256-thread build (solve3_p1.hip)
    if (grid && dim == 3) {
        switch (prec) {
            case IGA_PREC_FP64: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 0, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 0, 3, kBlock, 1>);
            case IGA_PREC_FP32: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 1, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 1, 3, kBlock, 1>);
            default: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 2, 3, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 2, 3, kBlock, 1>);
        }
    }
    if (grid) {
        switch (prec) {
            case IGA_PREC_FP64: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 0, 2, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 0, 2, kBlock, 1>);
            case IGA_PREC_FP32: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 1, 2, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 1, 2, kBlock, 1>);
            default: return grid == 2 ? reinterpret_cast<const void*>(k_solve_grid<1, 2, 2, kBlock, 2>)
                             : reinterpret_cast<const void*>(k_solve_grid<1, 2, 2, kBlock, 1>);
        }
    }
    if (dim == 3) {
        switch (prec) {
            case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<1, 0, 3, kBlock>);
            case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<1, 1, 3, kBlock>);
            default: return reinterpret_cast<const void*>(k_solve<1, 2, 3, kBlock>);
        }
    }
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<1, 0, 2, kBlock>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<1, 1, 2, kBlock>);
        default: return reinterpret_cast<const void*>(k_solve<1, 2, 2, kBlock>);
    }
}

}  // namespace igasg
