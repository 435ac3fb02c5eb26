// stp_plain_f32_rt.hip -- plain kernel, I/O type float and accumulator float, generic classes with a run-time quantity
// count m < 9 (bounds 4 and 9).
#include "stp_plain.hpp"

namespace stp {

KernelInfo plain_kernel_f32_rt4(int N) { return plain::plain_generic_rt<float, float, 4>(N); }
KernelInfo plain_kernel_f32_rt9(int N) { return plain::plain_generic_rt<float, float, 9>(N); }

}  // namespace stp
