// stp_launch.hip -- kernel selection and launch of a batch: one launch for a uniform batch, or for a
// heterogeneous batch a device-side bucketing pass (element lists per class, tile queues per bucket, no host
// synchronisation) followed by one persistent launch per physics bucket on the caller's stream, with the
// classes that have their own launch forked onto side streams and joined back with events.
#include <algorithm>
#include <mutex>

#include "stp_hetero.hpp"
#include "stp_plan.hpp"

namespace stp {

namespace {

__global__ void clear_counts(int32_t* counts, int n)
{
    int i = threadIdx.x;
    if (i < n) counts[i] = 0;
}

// Elements with a class id outside 0..nclass-1 are skipped (their outputs are not written) and flagged in
// *bad, which the host reports (stp_sync, or the serving ticket's status).
__global__ void bucket_by_class(const int32_t* cls, int64_t nelem, int nclass, int32_t* lists, int64_t cap,
                                int32_t* counts, int32_t* bad)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nelem) return;
    int c = cls[e];
    if (c < 0 || c >= nclass) {
        *bad = 1;
        return;
    }
    int pos = atomicAdd(&counts[c], 1);
    lists[(int64_t)c * cap + pos] = (int32_t)e;
}

// The three bucketing steps (clear, per-class lists, tile queues) in one workgroup with the counts in LDS, for
// batches small enough that one workgroup sorts them quickly: two launches fewer per batch (serving batches
// are a few hundred elements). Same outputs as clear_counts + bucket_by_class + hetero_setup (the order of the
// elements inside a class list is arbitrary in both).
constexpr int kBucketThreads = 1024;
constexpr int64_t kBucketSmallMax = 65536;

__global__ void __launch_bounds__(kBucketThreads)
    bucket_small(const int32_t* cls, int64_t nelem, int nclass, int32_t* lists, int64_t cap, int32_t* counts,
                 const int32_t* slots, const int32_t* orders, const int32_t* bncls, int32_t* tile_start, int32_t* heads,
                 int32_t* bad)
{
    __shared__ int32_t cnt[kMaxClasses];
    const int t = threadIdx.x;
    if (t < kMaxClasses) cnt[t] = 0;
    __syncthreads();
    for (int64_t e = t; e < nelem; e += kBucketThreads) {
        const int c = cls[e];
        if (c < 0 || c >= nclass) {  // skipped and flagged, as in bucket_by_class
            *bad = 1;
            continue;
        }
        const int pos = atomicAdd(&cnt[c], 1);
        lists[(int64_t)c * cap + pos] = (int32_t)e;
    }
    __syncthreads();
    if (t < nclass) counts[t] = cnt[t];
    if (t < kHeteroBuckets) {
        int acc = 0;
        const int nc = bncls[t];
        for (int k = 0; k < nc; ++k) {
            tile_start[t * (kMaxClasses + 1) + k] = acc;
            const int c = orders[t * kMaxClasses + k];
            acc += (cnt[c] + slots[c] - 1) / slots[c];
        }
        tile_start[t * (kMaxClasses + 1) + nc] = acc;
        heads[t] = 0;
    }
}

// Tile queues of the persistent kernel: for every bucket, the first tile of each class in processing order
// and a reset tile counter. One thread per bucket.
__global__ void hetero_setup(const int32_t* counts, const int32_t* slots, const int32_t* orders, const int32_t* bncls,
                             int32_t* tile_start, int32_t* heads)
{
    const int b = threadIdx.x;
    if (b >= kHeteroBuckets) return;
    int acc = 0;
    const int nc = bncls[b];
    for (int k = 0; k < nc; ++k) {
        tile_start[b * (kMaxClasses + 1) + k] = acc;
        const int c = orders[b * kMaxClasses + k];
        acc += (counts[c] + slots[c] - 1) / slots[c];
    }
    tile_start[b * (kMaxClasses + 1) + nc] = acc;
    heads[b] = 0;
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
    for (void* q : {(void*)s.lists, (void*)s.counts, (void*)s.tile_start, (void*)s.heads})
        if (q) (void)hipFree(q);
    for (int i = 0; i < kSideStreams; ++i) {
        if (s.side[i]) (void)hipStreamDestroy(s.side[i]);
        if (s.join[i]) (void)hipEventDestroy(s.join[i]);
    }
    if (s.fork) (void)hipEventDestroy(s.fork);
    s = HeteroScratch{};
}

namespace {

struct Eligibility {
    bool fused, mfma;
};

Eligibility eligible(const stp_plan_s* p, const ClassState& cs)
{
    // the fused kernel implements the Cartesian presets up to order 7; the split-BF16 MFMA kernels the Cartesian
    // presets at orders 7 to 9 and curvilinear elastic elements at order 7; the FP32 MFMA kernel the Cartesian
    // presets at order 7
    const bool cart = cs.cls.physics == STP_ACOUSTIC || cs.cls.physics == STP_ELASTIC;
    const bool curv = cs.cls.physics == STP_ELASTIC_CURV;
    const bool f32io = p->prec != STP_FP64;
    const bool simple = f32io && !cs.acc64 && !(cs.cls.flags & STP_SRC_POINT);
    const int N = cs.cls.order;
    return {simple && cart && N <= 7,
            simple && ((p->prec == STP_BF16X3 && ((N == 7 && (cart || curv)) || ((N == 8 || N == 9) && cart))) ||
                       (p->prec == STP_FP32 && N == 7 && cart))};
}

// Generic classes with dense per-node B_d and no other terms (no A, no point source), FP32 arithmetic and
// accumulation: the kernel that keeps B_d on chip through the Taylor loop, where one exists for the order and m.
KernelInfo resident_for(const stp_plan_s* p, const ClassState& cs)
{
    const unsigned other = STP_A_PRESENT | STP_SRC_POINT | STP_COEF_PER_ELEMENT;
    if (p->prec == STP_FP64 || cs.acc64 || cs.cls.physics != STP_GENERIC || (cs.cls.flags & other)) return {};
    return resident_kernel_f32(cs.cls.order, cs.cls.nquant);
}

// the plain variant: the on-chip B_d kernel where it applies, else the plain kernel
KernelInfo plain_for(const stp_plan_s* p, const ClassState& cs)
{
    const KernelInfo r = resident_for(p, cs);
    return r.fn ? r : plain_kernel(p->prec == STP_FP64, cs.acc64, cs.cls.order, cs.cls.physics, cs.cls.nquant);
}

// the matrix-core kernel of the plan's precision: FP32 products, or split-BF16 products with FP32 accumulation
KernelInfo mfma_for(const stp_plan_s* p, const ClassState& cs)
{
    return p->prec == STP_FP32 ? mfma32_kernel_n7(cs.cls.physics) : mfma_kernel(cs.cls.order, cs.cls.physics);
}

}  // namespace

std::vector<std::pair<int, KernelInfo>> kernel_candidates(stp_plan_s* p, const ClassState& cs)
{
    const Eligibility el = eligible(p, cs);
    std::vector<std::pair<int, KernelInfo>> v;
    v.push_back({STP_VARIANT_PLAIN, plain_for(p, cs)});
    if (el.fused) v.push_back({STP_VARIANT_FUSED, fused_kernel_f32(cs.cls.order, cs.cls.physics)});
    if (el.mfma) v.push_back({STP_VARIANT_MFMA, mfma_for(p, cs)});
    return v;
}

KernelInfo select_kernel(stp_plan_s* p, const ClassState& cs, int* variant)
{
    const Eligibility el = eligible(p, cs);
    const KernelInfo plain = plain_for(p, cs);
    int v = p->variant;
    if (v == STP_VARIANT_AUTO)  // built-in rule: matrix cores where a kernel exists, else fused, else plain
        v = el.mfma ? STP_VARIANT_MFMA : (el.fused ? STP_VARIANT_FUSED : STP_VARIANT_PLAIN);
    if (variant) *variant = v;
    switch (v) {
    case STP_VARIANT_PLAIN:
        return plain;
    case STP_VARIANT_FUSED:
        return el.fused ? fused_kernel_f32(cs.cls.order, cs.cls.physics) : KernelInfo{};
    case STP_VARIANT_MFMA:
        return el.mfma ? mfma_for(p, cs) : KernelInfo{};
    default:
        return KernelInfo{};
    }
}

stp_status reserve_scratch(stp_plan_s* p, HeteroScratch& s, int64_t nelem)
{
    const int nclass = (int)p->classes.size();
    if (s.cap >= nelem && s.counts) return STP_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    int32_t* const bad = s.bad;  // not owned by the scratch (a serving lane's flag word)
    free_scratch(s);
    s.bad = bad;
    const size_t cap = (size_t)std::max<int64_t>(nelem, 1);
    if ((e = hipMalloc(&s.lists, sizeof(int32_t) * (size_t)nclass * cap)) != hipSuccess) return hip_fail(e, "hipMalloc(lists)");
    if ((e = hipMalloc(&s.counts, sizeof(int32_t) * kMaxClasses)) != hipSuccess) return hip_fail(e, "hipMalloc(counts)");
    if ((e = hipMalloc(&s.tile_start, sizeof(int32_t) * kHeteroBuckets * (kMaxClasses + 1))) != hipSuccess)
        return hip_fail(e, "hipMalloc(tile_start)");
    if ((e = hipMalloc(&s.heads, sizeof(int32_t) * kHeteroBuckets)) != hipSuccess) return hip_fail(e, "hipMalloc(heads)");
    if ((e = hipEventCreateWithFlags(&s.fork, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    for (int i = 0; i < kSideStreams; ++i) {
        if ((e = hipStreamCreateWithFlags(&s.side[i], hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreate(side)");
        if ((e = hipEventCreateWithFlags(&s.join[i], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "hipEventCreate");
    }
    s.cap = (int64_t)cap;
    return STP_OK;
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
            // grow (synchronous allocation); stp_reserve makes this a no-op, as graph capture requires
            stp_status st = reserve_scratch(p, *s, b->nelem);
            if (st != STP_OK) return st;
        }
    }
    int32_t* bad = s->bad ? s->bad : p->d_bad;
    if (b->nelem <= kBucketSmallMax) {
        hipLaunchKernelGGL(bucket_small, dim3(1), dim3(kBucketThreads), 0, stream, b->cls, b->nelem, nclass, s->lists,
                           s->cap, s->counts, p->d_slots, p->d_orders, p->d_bncls, s->tile_start, s->heads, bad);
    } else {
        hipLaunchKernelGGL(clear_counts, dim3(1), dim3(64), 0, stream, s->counts, nclass);
        hipLaunchKernelGGL(bucket_by_class, dim3((unsigned)((b->nelem + 255) / 256)), dim3(256), 0, stream, b->cls,
                           b->nelem, nclass, s->lists, s->cap, s->counts, bad);
        hipLaunchKernelGGL(hetero_setup, dim3(1), dim3(64), 0, stream, s->counts, p->d_slots, p->d_orders,
                           p->d_bncls, s->tile_start, s->heads);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "bucketing launch");
    // classes with their own launch (high orders, FP64 accumulation or I/O), most expensive first
    std::vector<int> order;
    for (int c = 0; c < nclass; ++c)
        if (!p->classes[c].tiled) order.push_back(c);
    std::sort(order.begin(), order.end(), [&](int x, int y) { return p->classes[x].flops > p->classes[y].flops; });
    bool anyTiled = false;
    for (auto& bp : p->buckets) anyTiled |= !bp.order.empty();
    // With tiled classes present, the own-launch classes go to the side streams (fork after the setup pass).
    // Small batches stay on one stream: there the fork and join cost more than the overlap gains (serving
    // batches of a few hundred elements lost half their throughput).
    const bool fork = s->fork && anyTiled && !order.empty() && b->nelem >= kForkMinElements;
    const int nside = fork ? std::min<int>(kSideStreams, (int)order.size()) : 0;
    if (fork) {
        if ((e = hipEventRecord(s->fork, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord(fork)");
        for (int i = 0; i < nside; ++i)
            if ((e = hipStreamWaitEvent(s->side[i], s->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    for (size_t k = 0; k < order.size(); ++k) {
        const int c = order[k];
        const ClassState& cs = p->classes[c];
        StpArgs a = base_args(p, cs, b);
        a.list = s->lists + (int64_t)c * s->cap;
        a.count = s->counts + c;
        const int64_t grid = std::min<int64_t>(b->nelem, (int64_t)p->num_cus * 8);
        stp_status st = launch_one(cs, a, grid, fork ? s->side[k % nside] : stream);
        if (st != STP_OK) return st;
    }
    // one persistent launch per physics bucket for the tiled classes
    for (int bk = 0; bk < kHeteroBuckets; ++bk) {
        const BucketPlan& bp = p->buckets[bk];
        if (bp.order.empty()) continue;
        hetero::HArgs h{};
        h.a = base_args(p, p->classes[bp.order[0]], b);
        h.cls = static_cast<const hetero::HClass*>(p->d_hcls);
        h.lists = s->lists;
        h.cap = s->cap;
        h.counts = s->counts;
        h.order = p->d_orders + bk * kMaxClasses;
        h.tile_start = s->tile_start + bk * (kMaxClasses + 1);
        h.head = s->heads + bk;
        h.ncls = (int)bp.order.size();
        void* args[] = {&h};
        // never more workgroups than elements (a tile holds at least one)
        const int grid = (int)std::min<int64_t>((int64_t)p->num_cus * p->hetero_grid_per_cu, b->nelem);
        e = hipLaunchKernel(bp.kernel.fn, dim3(grid), dim3(bp.kernel.threads), args, bp.lds, stream);
        if (e != hipSuccess) return hip_fail(e, "hipLaunchKernel(heterogeneous)");
    }
    for (int i = 0; i < nside; ++i) {  // join: the caller's stream waits for the side streams
        if ((e = hipEventRecord(s->join[i], s->side[i])) != hipSuccess) return hip_fail(e, "hipEventRecord(join)");
        if ((e = hipStreamWaitEvent(stream, s->join[i], 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    return STP_OK;
}

stp_status hetero_prepare(stp_plan_s* p)
{
    const int nclass = (int)p->classes.size();
    for (void** q : {&p->d_hcls, (void**)&p->d_slots, (void**)&p->d_orders, (void**)&p->d_bncls, (void**)&p->d_bad})
        if (*q) {
            (void)hipFree(*q);
            *q = nullptr;
        }
    const size_t budget = p->hetero_lds_budget;
    p->buckets.assign(kHeteroBuckets, BucketPlan{});
    std::vector<hetero::HClass> hc(nclass);
    std::vector<int32_t> slots(nclass, 1), orders(kHeteroBuckets * kMaxClasses, 0), bncls(kHeteroBuckets, 0);
    const bool f32io = p->prec != STP_FP64;
    for (int c = 0; c < nclass; ++c) {
        ClassState& cs = p->classes[c];
        const int N = cs.cls.order, nn = (N + 1) * (N + 1) * (N + 1);
        const bool hasA = cs.cls.physics == STP_GENERIC && (cs.cls.flags & STP_A_PRESENT);
        cs.tiled = false;
        // tiles of the persistent launch; classes of the on-chip B_d kernel keep their own launch (a tile slot
        // has one thread per node and the LDS of a few elements, too little to hold B_d)
        if (f32io && !cs.acc64 && N <= hetero::kMaxOrder && !resident_for(p, cs).fn) {
            const int bk = hetero::bucket_of(cs.cls.physics, cs.cls.nquant);
            const HeteroKernel k = hetero_kernel_f32(bk);
            const size_t sl = k.fn ? k.slot_lds(N, cs.cls.nquant, hasA) : 0;
            if (k.fn && sl <= budget) {
                cs.tiled = true;
                cs.bucket = bk;
                cs.slot_lds = sl;
                cs.slots = (int)std::min<size_t>(k.threads / nn, budget / sl);
                p->buckets[bk].kernel = k;
                p->buckets[bk].order.push_back(c);
            }
        }
        hetero::HClass& h = hc[c];
        h.N = N;
        h.nn = nn;
        h.slots = cs.tiled ? cs.slots : 1;
        h.m = cs.cls.nquant;
        h.flags = cs.cls.flags;
        h.lds_slot = (unsigned)cs.slot_lds;
        h.size_q = cs.size_q;
        h.size_coef = cs.size_coef;
        h.size_face = cs.size_face;
        h.size_src = cs.size_src;
        h.D = cs.dD;  // the plain element routine reads the full derivative matrix
        h.e0 = cs.de0;
        h.e1 = cs.de1;
        slots[c] = h.slots;
    }
    for (int bk = 0; bk < kHeteroBuckets; ++bk) {
        BucketPlan& bp = p->buckets[bk];
        std::sort(bp.order.begin(), bp.order.end(),
                  [&](int x, int y) { return p->classes[x].flops > p->classes[y].flops; });
        bncls[bk] = (int32_t)bp.order.size();
        for (size_t k = 0; k < bp.order.size(); ++k) {
            orders[bk * kMaxClasses + k] = bp.order[k];
            const ClassState& cs = p->classes[bp.order[k]];
            bp.lds = std::max(bp.lds, cs.slot_lds * (size_t)cs.slots);
        }
        if (bp.lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(bp.kernel.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bp.lds);
            if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(heterogeneous LDS)");
        }
    }
    hipError_t e;
    if ((e = hipMalloc(&p->d_bad, sizeof(int32_t))) != hipSuccess) return hip_fail(e, "hipMalloc(flag)");
    if ((e = hipMemset(p->d_bad, 0, sizeof(int32_t))) != hipSuccess) return hip_fail(e, "hipMemset(flag)");
    if ((e = hipMalloc(&p->d_hcls, sizeof(hetero::HClass) * nclass)) != hipSuccess) return hip_fail(e, "hipMalloc(classes)");
    if ((e = hipMemcpy(p->d_hcls, hc.data(), sizeof(hetero::HClass) * nclass, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(classes)");
    if ((e = hipMalloc(&p->d_slots, sizeof(int32_t) * nclass)) != hipSuccess) return hip_fail(e, "hipMalloc(slots)");
    if ((e = hipMemcpy(p->d_slots, slots.data(), sizeof(int32_t) * nclass, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(slots)");
    if ((e = hipMalloc(&p->d_orders, sizeof(int32_t) * orders.size())) != hipSuccess) return hip_fail(e, "hipMalloc(orders)");
    if ((e = hipMemcpy(p->d_orders, orders.data(), sizeof(int32_t) * orders.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(orders)");
    if ((e = hipMalloc(&p->d_bncls, sizeof(int32_t) * kHeteroBuckets)) != hipSuccess) return hip_fail(e, "hipMalloc(bncls)");
    if ((e = hipMemcpy(p->d_bncls, bncls.data(), sizeof(int32_t) * kHeteroBuckets, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy(bncls)");
    return STP_OK;
}

}  // namespace stp

// ------------------------------------------------------------------------------------------------------------
// Static scratch of the no-allocation entry point. Callers that cannot allocate device memory (code under HIP
// graph capture, serving loops that forbid allocation) get the heterogeneous bucketing scratch from this
// file-scope device array instead of the plan's allocated scratch. Every device the library runs on holds its
// own copy until the process ends. Layout (int32 words): counts [kMaxClasses], tile_start
// [kHeteroBuckets][kMaxClasses + 1], heads [kHeteroBuckets], then the per-class element lists
// [nclass][nelem]. In host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device.
namespace stp {
namespace {

constexpr int64_t kStaticHeaderWords = 1024;                 // counts, tile queues, heads (4 KiB)
constexpr int64_t kStaticListWords = int64_t(4) << 20;       // per-class element lists (16 MiB)
static_assert(kMaxClasses + kHeteroBuckets * (kMaxClasses + 1) + kHeteroBuckets <= kStaticHeaderWords,
              "the bucketing header fits its region");

static __device__ __align__(256) int32_t scratch[kStaticHeaderWords + kStaticListWords];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
int32_t* g_static_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

stp_status static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(STP_E_UNSUPPORTED, "device %d >= %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_ptr[device]) return STP_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(static scratch)");
    g_static_ptr[device] = static_cast<int32_t*>(ptr);
    return STP_OK;
}

}  // namespace stp

extern "C" stp_status stp_run_noalloc(stp_plan_t p, const stp_batch* b, void* stream)
{
    using namespace stp;
    clear_last_error();
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    stp_status st = validate_batch(p, b);
    if (st != STP_OK) return st;
    if (b->nelem == 0) return STP_OK;
    const int64_t nclass = (int64_t)p->classes.size();
    if (nclass > 1 && nclass * b->nelem > kStaticListWords)
        return fail(STP_E_INVAL, "nclass * nelem = %lld exceeds the static scratch (%lld entries)",
                    (long long)(nclass * b->nelem), (long long)kStaticListWords);
    DeviceGuard g(p->device);
    if (nclass == 1) return launch_batch(p, b, static_cast<hipStream_t>(stream));  // no scratch in use
    int32_t* base;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        base = g_static_ptr[p->device];
    }
    if (!base) return fail(STP_E_DEVICE, "static scratch of device %d not resolved", p->device);
    // The bucketing kernels clear the counts and tile heads themselves (no memset); no side streams, so the
    // own-launch classes run on the caller's stream.
    HeteroScratch s{};
    s.counts = base;
    s.tile_start = base + kMaxClasses;
    s.heads = s.tile_start + kHeteroBuckets * (kMaxClasses + 1);
    s.lists = base + kStaticHeaderWords;
    s.cap = b->nelem;
    return launch_batch(p, b, static_cast<hipStream_t>(stream), &s);
}
