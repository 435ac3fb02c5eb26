// stp_hetero.hpp -- persistent launch for a batch of elements of mixed order, quantity count and physics.
//
// The host plan sorts its classes by per-element cost (largest first) and groups them by physics bucket (the
// register footprint of a class depends mostly on its quantity bound, so each bucket gets its own kernel).
// A device-side setup pass turns the per-class counts of the bucketing pass into a queue of tiles per bucket:
// a tile is up to `slots` elements of one class, processed together by a 512-thread workgroup with one
// thread per node (slot s uses threads [s n^3, (s+1) n^3)). Workgroups of the persistent grid take tiles
// from the queue with an atomic counter, so the expensive orders start first and cheap ones fill in behind;
// every tile dispatches on its order to the element routine of the plain kernel. Everything is launched on
// the caller's stream without host synchronisation or memsets, so a batch can be captured into a HIP graph.
// Covers orders 1..7 (n^3 <= 512); higher orders, and the generic classes whose kernel keeps B_d on chip, run as
// per-class launches of their own kernel.
#pragma once
#include <type_traits>

#include "stp_kernels.hpp"
#include "stp_plain.hpp"

namespace stp {
namespace hetero {

constexpr int kThreads = 512;
constexpr int kMaxOrder = 7;
constexpr int kBuckets = 4;

// Device descriptor of one class.
struct HClass {
    int N;
    int nn;             // nodes per element (threads per slot)
    int slots;          // elements per tile
    int m;
    unsigned flags;
    unsigned lds_slot;  // bytes of LDS per slot
    int64_t size_q, size_coef, size_face, size_src;
    const void* D;
    const void* e0;
    const void* e1;
};

struct HArgs {
    StpArgs a;                   // batch pointers (per-class fields are filled from HClass)
    const HClass* cls;           // [nclass of the plan]
    const int32_t* lists;        // [nclass][cap] element ids per class (bucketing pass)
    int64_t cap;
    const int32_t* counts;       // [nclass]
    const int32_t* order;        // [ncls] classes of this bucket in processing order
    const int32_t* tile_start;   // [ncls + 1] first tile of each of them
    int32_t* head;               // tile counter of this bucket (reset by the setup pass)
    int ncls;
};

// Buckets: 0 acoustic, 1 elastic, 2 generic m == 4, 3 generic m == 9; -1 (no tiling: the class keeps its own
// launch) for generic classes with another quantity count, whose run-time-m element routines would cost
// minutes of compile time per bucket for classes that are rare in practice.
__host__ __device__ inline int bucket_of(int physics, int m)
{
    if (physics == kAcoustic) return 0;
    if (physics == kElastic) return 1;
    if (physics == kElasticCurv) return -1;
    if (m == 4) return 2;
    if (m == 9) return 3;
    return -1;
}

template <int B>
struct BucketTraits {
    static constexpr int PHYS = B == 0 ? kAcoustic : (B == 1 ? kElastic : kGeneric);
    static constexpr int MB = (B == 0 || B == 2) ? 4 : 9;
    static constexpr bool EX = B == 2 || B == 3;
};

template <typename T, typename ACC, int B, int N>
using ElemK = plain::Plain<T, ACC, N, BucketTraits<B>::PHYS, BucketTraits<B>::MB, BucketTraits<B>::EX>;

// The element routine with its thread count fixed at n^3 (one thread per node of the slot).
template <typename T, typename ACC, int B, int N>
__device__ __attribute__((always_inline)) inline void run_elem(const StpArgs& a, const ElemRef& er, bool valid,
                                                               unsigned char* base, int ltid)
{
    constexpr int nn = (N + 1) * (N + 1) * (N + 1);
    __builtin_assume(ltid >= 0 && ltid < nn);
    [[clang::always_inline]] ElemK<T, ACC, B, N>::element(a, er, valid, base, ltid, nn);
}

// One tile: find its class, map the workgroup's threads onto the class's slots and run the element routine
// for the class's order. Each order's routine is instantiated with its thread count as a constant (with a run-
// time count the compiler cannot drop the idle-thread paths and the m = 9 routines spill).
template <typename T, typename ACC, int B>
__device__ __attribute__((always_inline)) inline void hetero_tile(const HArgs& h, int item, unsigned char* smem)
{
    int k = 0;
    while (h.tile_start[k + 1] <= item) ++k;
    const int c = h.order[k];
    const HClass hc = h.cls[c];
    const int tile = item - h.tile_start[k];
    const int slot = threadIdx.x / hc.nn;
    const int ltid = threadIdx.x - slot * hc.nn;
    const int64_t li = (int64_t)tile * hc.slots + slot;
    const bool valid = slot < hc.slots && li < h.counts[c];

    StpArgs a = h.a;
    a.D = hc.D;
    a.e0 = hc.e0;
    a.e1 = hc.e1;
    a.m = hc.m;
    a.flags = hc.flags;
    a.stride_q = hc.size_q;
    a.stride_coef = hc.size_coef;
    a.stride_face = hc.size_face;
    a.stride_src = hc.size_src;
    a.list = nullptr;
    a.count = nullptr;
    a.nelem = INT64_MAX;
    ElemRef er{};
    er.h = 1.0;
    if (valid) elem_ref(a, h.lists[(int64_t)c * h.cap + li], er);
    unsigned char* base = smem + (size_t)(slot < hc.slots ? slot : 0) * hc.lds_slot;
    switch (hc.N) {
    case 1: run_elem<T, ACC, B, 1>(a, er, valid, base, ltid); break;
    case 2: run_elem<T, ACC, B, 2>(a, er, valid, base, ltid); break;
    case 3: run_elem<T, ACC, B, 3>(a, er, valid, base, ltid); break;
    case 4: run_elem<T, ACC, B, 4>(a, er, valid, base, ltid); break;
    case 5: run_elem<T, ACC, B, 5>(a, er, valid, base, ltid); break;
    case 6: run_elem<T, ACC, B, 6>(a, er, valid, base, ltid); break;
    default: run_elem<T, ACC, B, 7>(a, er, valid, base, ltid); break;
    }
}

template <typename T, typename ACC, int B>
__global__ void __launch_bounds__(kThreads) stp_hetero_kernel(HArgs h)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    const int total = h.tile_start[h.ncls];
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(h.head, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();  // every thread has read the item before thread 0 takes the next one
        if (item >= total) break;
        hetero_tile<T, ACC, B>(h, item, smem);
    }
}

// LDS bytes of one slot (16-byte multiple) for order N, quantity count m and optional A, in bucket B.
template <typename T, typename ACC, int B>
size_t slot_lds(int N, int m, bool hasA)
{
    size_t r = 0;
    switch (N) {
    case 1: r = ElemK<T, ACC, B, 1>::layout(m, hasA).total; break;
    case 2: r = ElemK<T, ACC, B, 2>::layout(m, hasA).total; break;
    case 3: r = ElemK<T, ACC, B, 3>::layout(m, hasA).total; break;
    case 4: r = ElemK<T, ACC, B, 4>::layout(m, hasA).total; break;
    case 5: r = ElemK<T, ACC, B, 5>::layout(m, hasA).total; break;
    case 6: r = ElemK<T, ACC, B, 6>::layout(m, hasA).total; break;
    case 7: r = ElemK<T, ACC, B, 7>::layout(m, hasA).total; break;
    default: break;
    }
    return (r + 15) & ~size_t(15);
}

template <int B>
HeteroKernel hetero_info()
{
    HeteroKernel k;
    k.fn = reinterpret_cast<const void*>(&stp_hetero_kernel<float, float, B>);
    k.slot_lds = &slot_lds<float, float, B>;
    k.threads = kThreads;
    k.max_order = kMaxOrder;
    return k;
}

}  // namespace hetero
}  // namespace stp
