// stp_hetero_b0.hip -- the heterogeneous persistent kernel of physics bucket 0 (FP32).
#include "stp_hetero.hpp"

namespace stp {

HeteroKernel hetero_kernel_f32_b0() { return hetero::hetero_info<0>(); }

}  // namespace stp
