// stp_mfma_n7.hip -- instantiations of the split-BF16 MFMA preset kernel (order 7).
#include "stp_mfma.hpp"

namespace stp {

KernelInfo mfma_kernel_n7(int physics)
{
    if (physics == kElastic) return mfma::mfma_info<kElastic>();
    if (physics == kAcoustic) return mfma::mfma_info<kAcoustic>();
    if (physics == kElasticCurv) return mfma::mfma_info<kElasticCurv>();
    return KernelInfo{};
}

}  // namespace stp
