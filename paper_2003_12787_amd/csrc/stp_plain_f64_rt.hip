// stp_plain_f64_rt.hip -- plain kernel, I/O type double and accumulator double, generic classes with a run-time quantity
// count m < 9 (bounds 4 and 9).
#include "stp_plain.hpp"

namespace stp {

KernelInfo plain_kernel_f64_rt4(int N) { return plain::plain_generic_rt<double, double, 4>(N); }
KernelInfo plain_kernel_f64_rt9(int N) { return plain::plain_generic_rt<double, double, 9>(N); }

}  // namespace stp
