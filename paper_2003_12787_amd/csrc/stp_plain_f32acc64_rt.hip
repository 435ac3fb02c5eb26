// stp_plain_f32acc64_rt.hip -- plain kernel, I/O type float and accumulator double, generic classes with a run-time quantity
// count m < 9 (bounds 4 and 9).
#include "stp_plain.hpp"

namespace stp {

KernelInfo plain_kernel_f32acc64_rt4(int N) { return plain::plain_generic_rt<float, double, 4>(N); }
KernelInfo plain_kernel_f32acc64_rt9(int N) { return plain::plain_generic_rt<float, double, 9>(N); }

}  // namespace stp
