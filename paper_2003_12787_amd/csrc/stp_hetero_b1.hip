// stp_hetero_b1.hip -- the heterogeneous persistent kernel of physics bucket 1 (FP32).
#include "stp_hetero.hpp"

namespace stp {

HeteroKernel hetero_kernel_f32_b1() { return hetero::hetero_info<1>(); }

}  // namespace stp
