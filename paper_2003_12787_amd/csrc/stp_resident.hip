// stp_resident.hip -- instantiations of the kernel with on-chip B_d (generic classes, dense per-node B_d: m = 4
// at orders 4 to 9, m = 9 at orders 7 to 9). Per order: threads per workgroup, nodes per thread, the words of
// each node's B_d held in registers and in LDS, and the derivative grouping. Every choice compiles without
// spills at the waves per SIMD of its thread count and was the fastest of those timed for its class:
//  - m = 9: one node per thread keeps the waves (and the loads in flight) of the plain kernel while the LDS
//    beside the element's tiles holds part of B_d, and the registers left under the thread count's cap hold a
//    few more words (N = 8: 20, 6% faster than none); at N = 9 two nodes per thread with 24 words in
//    registers measured 3% faster. At N = 7 the next column's streamed words are loaded before the current
//    column's derivative (two columns of loads in flight): 0.573 to 0.541 ms; at N = 8 and 9 it measured the
//    same, and with fewer register words to make room for it, 2-4% slower. Derivatives one quantity at a time: forming four together (16-byte LDS reads) needs a
//    padded tile, so fewer LDS-resident words, and measured 2-4% slower at N = 7 and 8.
//  - m = 4: all 48 words in registers, four derivatives together (1.5x to 2.2x faster than one at a time, and
//    about 2x faster than the tiled persistent launch at orders 4 to 6).
// For m = 9 below order 7 the on-chip variants measured slower than the tiled persistent launch (the whole
// B_d of an element fits on chip only at one wave per SIMD; LDS-resident words alone, at one workgroup per CU,
// took order 6 from 0.36 to 0.47 ms), so those classes keep it.
#include "stp_resident.hpp"

namespace stp {

KernelInfo resident_kernel_f32(int N, int m)
{
    using namespace resident;
    if (m == 9) {
        switch (N) {
        case 7: return resident_info<7, 9, 512, 1, 64, 70, 1, true>();   // 134 of 243 words on chip
        case 8: return resident_info<8, 9, 768, 1, 20, 47>();   // 67
        case 9: return resident_info<9, 9, 512, 2, 24, 31>();   // 55
        default: return KernelInfo{};
        }
    }
    if (m == 4) {  // all 48 words on chip
        switch (N) {
        case 4: return resident_info<4, 4, 128, 1, 48, 0, 4>();
        case 5: return resident_info<5, 4, 256, 1, 48, 0, 4>();
        case 6: return resident_info<6, 4, 384, 1, 48, 0, 4>();
        case 7: return resident_info<7, 4, 512, 1, 48, 0, 4>();
        case 8: return resident_info<8, 4, 768, 1, 48, 0, 4>();
        case 9: return resident_info<9, 4, 512, 2, 48, 0, 4>();
        default: return KernelInfo{};
        }
    }
    return KernelInfo{};
}

}  // namespace stp
