// stp_hetero_b5.hip -- the heterogeneous persistent kernel of physics bucket 5 (FP32).
#include "stp_hetero.hpp"

namespace stp {

HeteroKernel hetero_kernel_f32_b5() { return hetero::hetero_info<5>(); }

}  // namespace stp
