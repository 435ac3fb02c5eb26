// stp_mfma_f32_n7.hip -- instantiations of the FP32 MFMA preset kernel (order 7).
#include "stp_mfma_f32.hpp"

namespace stp {

KernelInfo mfma32_kernel_n7(int physics)
{
    if (physics == kElastic) return mfma32::mfma32_info<kElastic>();
    if (physics == kAcoustic) return mfma32::mfma32_info<kAcoustic>();
    return KernelInfo{};
}

}  // namespace stp
