// stp_plain_f32acc64.hip -- instantiations of the plain kernel with I/O type float and accumulator double: presets and the
// generic classes with m = 4 or 9; other generic quantity counts are in stp_plain_f32acc64_rt*.hip.
#include "stp_plain.hpp"

namespace stp {

KernelInfo plain_kernel_f32acc64(int N, int physics, int m)
{
    if (physics != kGeneric || m == 4 || m == 9) return plain::plain_by_physics<float, double>(N, physics, m);
    if (m < 4) return plain_kernel_f32acc64_rt4(N);
    if (m < 9) return plain_kernel_f32acc64_rt9(N);
    return plain_kernel_f32acc64_rt16(N);
}

}  // namespace stp
