// stp_mfma_n89.hip -- instantiations of the split-BF16 MFMA preset kernel at orders 8 and 9.
#include "stp_mfma_hi.hpp"

namespace stp {

KernelInfo mfma_kernel_n89(int N, int physics)
{
    if (N == 8 && physics == kElastic) return mfma::mfma_hi_info<kElastic, 8>();
    if (N == 8 && physics == kAcoustic) return mfma::mfma_hi_info<kAcoustic, 8>();
    if (N == 9 && physics == kElastic) return mfma::mfma_hi_info<kElastic, 9>();
    if (N == 9 && physics == kAcoustic) return mfma::mfma_hi_info<kAcoustic, 9>();
    return KernelInfo{};
}

}  // namespace stp
