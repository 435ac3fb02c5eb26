// stp_launch.hip -- kernel selection and launch of a batch: one launch for a uniform batch, or for a
// heterogeneous batch a device-side bucketing pass (element lists per class, no host synchronisation)
// followed by one persistent-grid launch per class, all on the caller's stream.
#include <algorithm>

#include "stp_plan.hpp"

namespace stp {

namespace {

__global__ void clear_counts(int32_t* counts, int n)
{
    int i = threadIdx.x;
    if (i < n) counts[i] = 0;
}

__global__ void bucket_by_class(const int32_t* cls, int64_t nelem, int nclass, int32_t* lists, int64_t cap,
                                int32_t* counts)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nelem) return;
    int c = cls[e];
    if (c < 0 || c >= nclass) return;  // elements with an invalid class id are skipped
    int pos = atomicAdd(&counts[c], 1);
    lists[(int64_t)c * cap + pos] = (int32_t)e;
}

StpArgs base_args(const stp_plan_s* p, const ClassState& cs, const stp_batch* b)
{
    StpArgs a{};
    a.nelem = b->nelem;
    a.off_q = b->off_q;
    a.off_coef = b->off_coef;
    a.off_face = b->off_face;
    a.off_src = b->off_src;
    a.stride_q = cs.size_q;
    a.stride_coef = cs.size_coef;
    a.stride_face = cs.size_face;
    a.stride_src = cs.size_src;
    if (b->dt_h_scalar) {
        a.dt_s = b->dt[0];
        a.h_s = b->h[0];
    } else {
        a.dt = b->dt;
        a.h = b->h;
    }
    a.Q = b->Q;
    a.params = b->params;
    a.A = b->A;
    a.B = b->B;
    a.src = b->src;
    a.qavg = b->qavg;
    a.favg = b->favg;
    a.qface = b->qface;
    a.fface = b->fface;
    a.D = cs.kernel.aux == KernelInfo::kAuxEvenOdd ? cs.daux : cs.dD;
    a.e0 = cs.de0;
    a.e1 = cs.de1;
    a.Dsplit = cs.dDsplit;
    a.m = cs.cls.nquant;
    a.flags = cs.cls.flags;
    (void)p;
    return a;
}

stp_status launch_one(const ClassState& cs, StpArgs& a, int64_t grid, hipStream_t stream)
{
    void* args[] = {&a};
    hipError_t e = hipLaunchKernel(cs.kernel.fn, dim3((unsigned)grid), dim3(cs.kernel.block), args, cs.lds, stream);
    if (e != hipSuccess) return hip_fail(e, "hipLaunchKernel");
    return STP_OK;
}

}  // namespace

void free_scratch(HeteroScratch& s)
{
    if (s.lists) (void)hipFree(s.lists);
    if (s.counts) (void)hipFree(s.counts);
    s = HeteroScratch{};
}

KernelInfo select_kernel(stp_plan_s* p, const ClassState& cs)
{
    const bool preset = cs.cls.physics != STP_GENERIC;
    const bool f32io = p->prec != STP_FP64;
    const bool simple = preset && f32io && !cs.acc64 && !(cs.cls.flags & STP_SRC_POINT);
    const bool fused_ok = simple && cs.cls.order <= 7;
    const bool mfma_ok = simple && cs.cls.order == 7 && p->prec == STP_BF16X3;
    const KernelInfo plain = plain_kernel(p->prec == STP_FP64, cs.acc64, cs.cls.order, cs.cls.physics, cs.cls.nquant);
    switch (p->variant) {
    case STP_VARIANT_PLAIN:
        return plain;
    case STP_VARIANT_FUSED:
        return fused_ok ? fused_kernel_f32(cs.cls.order, cs.cls.physics) : KernelInfo{};
    case STP_VARIANT_MFMA:
        return mfma_ok ? mfma_kernel_n7(cs.cls.physics) : KernelInfo{};
    default:
        // split-BF16 plans use the matrix cores where a kernel exists and the FP32 kernels elsewhere
        if (mfma_ok) return mfma_kernel_n7(cs.cls.physics);
        if (fused_ok) return fused_kernel_f32(cs.cls.order, cs.cls.physics);
        return plain;
    }
}

stp_status launch_batch(stp_plan_s* p, const stp_batch* b, hipStream_t stream, HeteroScratch* scratch)
{
    const int nclass = (int)p->classes.size();
    if (nclass == 1) {
        const ClassState& cs = p->classes[0];
        StpArgs a = base_args(p, cs, b);
        const int64_t grid = std::min<int64_t>(b->nelem, INT32_MAX) / cs.kernel.elems_per_block +
                             (b->nelem % cs.kernel.elems_per_block != 0);
        return launch_one(cs, a, grid, stream);
    }
    HeteroScratch* s = scratch ? scratch : &p->run_scratch;
    {
        std::lock_guard<std::mutex> lk(p->run_mu);
        if (s->cap < b->nelem || !s->counts) {
            // grow (synchronous allocation; a plan reused with batches of at most this size never reallocates)
            hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            free_scratch(*s);
            e = hipMalloc(&s->lists, sizeof(int32_t) * (size_t)nclass * (size_t)b->nelem);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(lists)");
            e = hipMalloc(&s->counts, sizeof(int32_t) * kMaxClasses);
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(counts)");
            s->cap = b->nelem;
        }
    }
    hipLaunchKernelGGL(clear_counts, dim3(1), dim3(64), 0, stream, s->counts, nclass);
    hipLaunchKernelGGL(bucket_by_class, dim3((unsigned)((b->nelem + 255) / 256)), dim3(256), 0, stream, b->cls,
                       b->nelem, nclass, s->lists, s->cap, s->counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "bucket_by_class launch");
    // most expensive classes first so that they start while cheaper ones fill in behind
    std::vector<int> order(nclass);
    for (int c = 0; c < nclass; ++c) order[c] = c;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return p->classes[x].flops > p->classes[y].flops; });
    for (int c : order) {
        const ClassState& cs = p->classes[c];
        StpArgs a = base_args(p, cs, b);
        a.list = s->lists + (int64_t)c * s->cap;
        a.count = s->counts + c;
        const int64_t grid = std::min<int64_t>(b->nelem, (int64_t)p->num_cus * 8);
        stp_status st = launch_one(cs, a, grid, stream);
        if (st != STP_OK) return st;
    }
    return STP_OK;
}

}  // namespace stp
