// stp_resident.hip -- instantiations of the kernel with on-chip B_d (generic classes, dense per-node B_d, orders
// 7 to 9, m = 4 or 9). Per order: threads per workgroup, nodes per thread, and the words of each node's B_d held
// in registers and in LDS. Every choice compiles without spills at the waves per SIMD of its thread count, and
// was the fastest of those timed for its class. One node per thread keeps the waves (and the loads in flight)
// of the plain kernel while the LDS beside the element's tiles holds part of B_d; m = 4 fits whole in the
// registers. At N = 9, m = 9 two nodes per thread with 24 words in registers measured 3% faster. At orders 5
// and 6 the on-chip variants measured slower than the tiled persistent launch (B_d of a whole element fits only
// at one wave per SIMD), so those classes keep it.
#include "stp_resident.hpp"

namespace stp {

KernelInfo resident_kernel_f32(int N, int m)
{
    using namespace resident;
    if (m == 9) {
        switch (N) {
        case 7: return resident_info<7, 9, 512, 1, 64, 70>();   // 134 of 243 words on chip
        case 8: return resident_info<8, 9, 768, 1, 0, 47>();    // 47
        case 9: return resident_info<9, 9, 512, 2, 24, 31>();   // 55
        default: return KernelInfo{};
        }
    }
    if (m == 4) {
        switch (N) {
        case 7: return resident_info<7, 4, 512, 1, 48, 0>();    // all 48 words
        case 8: return resident_info<8, 4, 768, 1, 48, 0>();
        case 9: return resident_info<9, 4, 1024, 1, 48, 0>();
        default: return KernelInfo{};
        }
    }
    return KernelInfo{};
}

}  // namespace stp
