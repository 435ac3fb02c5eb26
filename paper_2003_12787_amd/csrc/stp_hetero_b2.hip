// stp_hetero_b2.hip -- the heterogeneous persistent kernel of physics bucket 2 (FP32).
#include "stp_hetero.hpp"

namespace stp {

HeteroKernel hetero_kernel_f32_b2() { return hetero::hetero_info<2>(); }

}  // namespace stp
