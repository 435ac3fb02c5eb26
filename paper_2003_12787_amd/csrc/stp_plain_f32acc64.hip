// stp_plain_f32acc64.hip -- instantiations of the plain kernel with I/O type float and accumulator double.
#include "stp_plain.hpp"

namespace stp {

KernelInfo plain_kernel_f32acc64(int N, int physics, int m) { return plain::plain_by_physics<float, double>(N, physics, m); }

}  // namespace stp
