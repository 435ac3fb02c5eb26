// stp_hetero_select.cpp -- bucket -> heterogeneous kernel.
#include "stp_kernels.hpp"

namespace stp {

HeteroKernel hetero_kernel_f32_b0();
HeteroKernel hetero_kernel_f32_b1();
HeteroKernel hetero_kernel_f32_b2();
HeteroKernel hetero_kernel_f32_b3();

HeteroKernel hetero_kernel_f32(int bucket)
{
    switch (bucket) {
    case 0: return hetero_kernel_f32_b0();
    case 1: return hetero_kernel_f32_b1();
    case 2: return hetero_kernel_f32_b2();
    case 3: return hetero_kernel_f32_b3();
    default: return HeteroKernel{};
    }
}

}  // namespace stp
