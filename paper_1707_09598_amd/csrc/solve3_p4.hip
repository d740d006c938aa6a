// solve3_p4.hip -- k_solve for spline degree 4 in 3D, each inner precision,
// built with 256-thread workgroups (see IGASG_THREADS in common.hpp).
#define IGASG_THREADS 256
#include "solve.hpp"

namespace igasg {

const void* solve3_kernel_p4(int prec) {
    switch (prec) {
        case IGA_PREC_FP64: return reinterpret_cast<const void*>(k_solve<4, 0, 3, kBlock>);
        case IGA_PREC_FP32: return reinterpret_cast<const void*>(k_solve<4, 1, 3, kBlock>);
        default: return reinterpret_cast<const void*>(k_solve<4, 2, 3, kBlock>);
    }
}

}  // namespace igasg
