// stp_hetero_b4.hip -- the heterogeneous persistent kernel of physics bucket 4 (FP32).
#include "stp_hetero.hpp"

namespace stp {

HeteroKernel hetero_kernel_f32_b4() { return hetero::hetero_info<4>(); }

}  // namespace stp
