// stp_plain_f64_rt16.hip -- plain kernel, I/O type double and accumulator double, generic classes with a run-time quantity
// count 9 < m <= 16.
#include "stp_plain.hpp"

namespace stp {

KernelInfo plain_kernel_f64_rt16(int N) { return plain::plain_generic_rt<double, double, 16>(N); }

}  // namespace stp
