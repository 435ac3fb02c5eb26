// stp_hetero_b6.hip -- the heterogeneous persistent kernel of physics bucket 6 (FP32).
#include "stp_hetero.hpp"

namespace stp {

HeteroKernel hetero_kernel_f32_b6() { return hetero::hetero_info<6>(); }

}  // namespace stp
