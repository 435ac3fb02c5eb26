// stp_hetero_b3.hip -- the heterogeneous persistent kernel of physics bucket 3 (FP32).
#include "stp_hetero.hpp"

namespace stp {

HeteroKernel hetero_kernel_f32_b3() { return hetero::hetero_info<3>(); }

}  // namespace stp
