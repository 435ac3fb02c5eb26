// stp_fused_f32.hip -- FP32 instantiations of the fused preset kernel (orders 1..7).
#include "stp_fused.hpp"

namespace stp {

KernelInfo fused_kernel_f32(int N, int physics)
{
    if (physics == kElastic) return fused::fused_by_order<float, kElastic>(N);
    if (physics == kAcoustic) return fused::fused_by_order<float, kAcoustic>(N);
    return KernelInfo{};
}

}  // namespace stp
