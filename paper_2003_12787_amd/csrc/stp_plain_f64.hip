// stp_plain_f64.hip -- instantiations of the plain kernel with I/O type double and accumulator double.
#include "stp_plain.hpp"

namespace stp {

KernelInfo plain_kernel_f64(int N, int physics, int m) { return plain::plain_by_physics<double, double>(N, physics, m); }

}  // namespace stp
