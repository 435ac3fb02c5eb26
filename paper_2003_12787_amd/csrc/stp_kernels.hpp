// stp_kernels.hpp -- host-visible descriptors of the predictor's kernel instantiations.
#pragma once
#include <cstddef>

#include "stp_device.hpp"

namespace stp {

struct KernelInfo {
    enum Aux { kAuxNone = 0, kAuxEvenOdd = 1, kAuxMfmaSplit = 2 };  // which derivative table the kernel reads through StpArgs::D
    const void* fn = nullptr;               // __global__ function, launched with one StpArgs argument
    int block = 0;                          // threads per workgroup
    int mb = 0;                             // register bound on the quantity count
    int elems_per_block = 1;                // elements processed per workgroup iteration
    size_t (*lds)(int m, bool hasA) = nullptr;  // dynamic LDS bytes per workgroup
    int aux = kAuxNone;
};

// Plain kernel (any class): FP64, or FP32 I/O with FP32 or FP64 accumulation.
KernelInfo plain_kernel_f64(int N, int physics, int m);
KernelInfo plain_kernel_f32(int N, int physics, int m);
KernelInfo plain_kernel_f32acc64(int N, int physics, int m);
// generic classes with a run-time quantity count, bounded by 4, 9 or 16
KernelInfo plain_kernel_f64_rt4(int N);
KernelInfo plain_kernel_f64_rt9(int N);
KernelInfo plain_kernel_f64_rt16(int N);
KernelInfo plain_kernel_f32_rt4(int N);
KernelInfo plain_kernel_f32_rt9(int N);
KernelInfo plain_kernel_f32_rt16(int N);
KernelInfo plain_kernel_f32acc64_rt4(int N);
KernelInfo plain_kernel_f32acc64_rt9(int N);
KernelInfo plain_kernel_f32acc64_rt16(int N);
// Fused kernel (presets, FP32, N <= 7): lanes own x-lines, even/odd derivatives, LDS transposes.
KernelInfo fused_kernel_f32(int N, int physics);

// Split-BF16 MFMA kernels (FP32 I/O): presets and curvilinear elastic at N = 7, Cartesian presets at N = 8, 9.
KernelInfo mfma_kernel_n7(int physics);
KernelInfo mfma_kernel_n89(int N, int physics);
inline KernelInfo mfma_kernel(int N, int physics) { return N == 7 ? mfma_kernel_n7(physics) : mfma_kernel_n89(N, physics); }
// FP32 MFMA kernel (FP32 I/O and arithmetic): Cartesian presets at N = 7.
KernelInfo mfma32_kernel_n7(int physics);

// Generic classes with dense per-node B_d, no A and no point source (FP32 I/O and arithmetic), with B_d held
// on chip through the Taylor loop: m = 4 at orders 4..9, m = 9 at orders 7..9; fn == nullptr elsewhere.
KernelInfo resident_kernel_f32(int N, int m);

// Heterogeneous persistent kernel of one physics bucket (FP32 I/O, orders 1..7, 512 threads per workgroup).
struct HeteroKernel {
    const void* fn = nullptr;
    size_t (*slot_lds)(int N, int m, bool hasA) = nullptr;
    int threads = 0;
    int max_order = 0;
};
HeteroKernel hetero_kernel_f32(int bucket);

inline KernelInfo plain_kernel(int prec_fp64, int acc64, int N, int physics, int m)
{
    if (prec_fp64) return plain_kernel_f64(N, physics, m);
    return acc64 ? plain_kernel_f32acc64(N, physics, m) : plain_kernel_f32(N, physics, m);
}

}  // namespace stp
