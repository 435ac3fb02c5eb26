// stp_plain_f32.hip -- instantiations of the plain kernel with I/O type float and accumulator float.
#include "stp_plain.hpp"

namespace stp {

KernelInfo plain_kernel_f32(int N, int physics, int m) { return plain::plain_by_physics<float, float>(N, physics, m); }

}  // namespace stp
