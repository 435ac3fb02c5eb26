// stp_plan.hpp -- internal state of a plan (the opaque stp_plan_t of stp.h).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "stp.h"
#include "stp_kernels.hpp"

namespace stp {

constexpr int kMaxClasses = 64;
constexpr int kHeteroBuckets = 4;
constexpr size_t kHeteroLdsBudget = 80 * 1024;  // per workgroup of the persistent kernel (two per CU)
constexpr size_t kMaxLds = 160 * 1024;

struct ClassState {
    stp_class cls{};
    void* dD = nullptr;      // derivative matrix in the compute precision
    void* de0 = nullptr;     // face vectors in the compute precision
    void* de1 = nullptr;
    void* de0_64 = nullptr;  // FP64 face vectors (FP32 plans)
    void* de1_64 = nullptr;
    void* dDsplit = nullptr; // BF16 three-piece split tables of D (split-BF16x3 variant)
    void* daux = nullptr;    // even/odd derivative tables in the compute precision (fused variant)
    void* dw = nullptr;      // Gauss-Legendre weights on [0, 1] in the compute precision (corrector)
    bool acc64 = false;      // FP64 accumulation of q-bar and faces
    KernelInfo kernel;
    int variant = 0;                               // STP_VARIANT_* of `kernel`
    std::vector<std::pair<int, KernelInfo>> cands; // kernels that exist for this class (variant, kernel)
    size_t lds = 0;
    double bytes = 0, flops = 0;  // algorithmic cost per element
    int64_t size_q = 0, size_face = 0, size_coef = 0, size_src = 0;  // values per element
    // heterogeneous plans: processed as tiles of the persistent bucket kernel, or by its own launch
    bool tiled = false;
    int bucket = -1;
    int slots = 0;        // elements per tile
    size_t slot_lds = 0;  // LDS bytes per slot
};

// One physics bucket of the persistent heterogeneous kernel.
struct BucketPlan {
    std::vector<int> order;  // tiled classes of the bucket, most expensive first
    HeteroKernel kernel;
    size_t lds = 0;          // dynamic LDS of a workgroup (largest tile of the bucket)
};

// Device scratch of heterogeneous launches: per-class element lists and counts.
constexpr int kSideStreams = 4;
constexpr int64_t kForkMinElements = 8192;  // heterogeneous batches at least this large use the side streams

struct HeteroScratch {
    int32_t* lists = nullptr;       // [nclass][cap]
    int32_t* counts = nullptr;      // [kMaxClasses]
    int32_t* tile_start = nullptr;  // [kHeteroBuckets][kMaxClasses + 1]
    int32_t* heads = nullptr;       // [kHeteroBuckets]
    int32_t* bad = nullptr;         // set to 1 by the bucketing pass when a class id is out of range (NULL:
                                    // the plan's d_bad)
    int64_t cap = 0;
    // Classes with their own launch run on side streams, forked from and joined back into the caller's
    // stream with events, concurrently with the persistent launches (their tails overlap).
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
};

struct ServeState;

}  // namespace stp

struct stp_plan_s {
    int device = 0;
    int prec = STP_FP64;
    int acc64_min_order = 0;
    int variant = 0;
    int num_cus = 256;
    size_t serve_budget = 0;
    std::vector<stp::ClassState> classes;
    std::mutex run_mu;         // guards `run_scratch` growth
    stp::HeteroScratch run_scratch;
    // heterogeneous plans
    std::vector<stp::BucketPlan> buckets;
    void* d_hcls = nullptr;       // hetero::HClass[nclass]
    int32_t* d_slots = nullptr;   // [nclass] elements per tile (1 for classes with their own launch)
    int32_t* d_orders = nullptr;  // [kHeteroBuckets][kMaxClasses]
    int32_t* d_bncls = nullptr;   // [kHeteroBuckets]
    int32_t* d_bad = nullptr;     // set to 1 when stp_run / stp_run_noalloc met an out-of-range class id
                                  // (read and cleared by stp_sync)
    int hetero_grid_per_cu = 4;   // persistent workgroups per CU
    size_t hetero_lds_budget = stp::kHeteroLdsBudget;  // LDS of one persistent workgroup (sets tile sizes)
    int autotune = 0;
    int nodes = 0;  // 0 Gauss-Legendre, 1 Gauss-Lobatto
    stp::ServeState* serve = nullptr;
};

namespace stp {

// Makes the plan's device current for the scope (restores the previous one if it changed).
struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) changed = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (changed && prev >= 0) (void)hipSetDevice(prev);
    }
};

stp_status fail(stp_status st, const char* fmt, ...);
void clear_last_error();
stp_status hip_fail(hipError_t e, const char* what);
void class_cost(const stp_class& c, int io_bytes, double* bytes, double* flops);
stp_status validate_batch(stp_plan_s* p, const stp_batch* b);
KernelInfo select_kernel(stp_plan_s* p, const ClassState& cs, int* variant = nullptr);
// Kernels that exist for the class under the plan's precision (variant id, kernel).
std::vector<std::pair<int, KernelInfo>> kernel_candidates(stp_plan_s* p, const ClassState& cs);
// Make `k` the class's kernel (LDS size and attribute).
stp_status set_kernel(stp_plan_s* p, ClassState& cs, const KernelInfo& k);
// Plan-time autotuning with the JSON cache (mode: 0 cache only, 1 tune what is missing, 2 retune).
stp_status autotune_plan(stp_plan_s* p, int mode);
// Queue the kernels of a validated, non-empty batch on `stream`, using `scratch` for heterogeneous lists.
stp_status launch_batch(stp_plan_s* p, const stp_batch* b, hipStream_t stream, HeteroScratch* scratch = nullptr);
// Plan-time set-up of the heterogeneous path (class tiling, buckets, device descriptors).
stp_status hetero_prepare(stp_plan_s* p);
// Make `s` hold batches of up to nelem elements (synchronous allocation).
stp_status reserve_scratch(stp_plan_s* p, HeteroScratch& s, int64_t nelem);
void free_scratch(HeteroScratch& s);
// Resolve, once per device and with that device current, the device address of the library's static scratch
// (the no-allocation entry point stp_run_noalloc); called at plan creation.
stp_status static_scratch_init(int device);
stp_status serve_start(stp_plan_s* p);
void serve_stop(stp_plan_s* p);
double now_seconds();

}  // namespace stp
