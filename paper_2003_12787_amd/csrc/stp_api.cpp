// stp_api.cpp -- the C ABI of libstp.so (declared in include/stp.h): plans, argument validation, kernel
// dispatch for uniform and heterogeneous batches, the algorithmic cost model, and error reporting.
// The serving runtime behind stp_submit / stp_poll lives in stp_serve.cpp.
#include "stp_plan.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "basis.hpp"
#include "mfma_tables.hpp"

namespace stp {

thread_local std::string g_last_error;

stp_status fail(stp_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_last_error() { g_last_error.clear(); }

stp_status hip_fail(hipError_t e, const char* what)
{
    return fail(STP_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

namespace {


int param_count(int physics) { return physics == STP_ACOUSTIC ? 2 : (physics == STP_ELASTIC ? 3 : 12); }

int quantities_read(const stp_class& c, int d)
{
    (void)d;
    if (c.physics == STP_ACOUSTIC) return 2;  // p and v_d
    if (c.physics == STP_ELASTIC) return 6;   // three velocities and three stresses s_{d,i}
    return c.nquant;                          // generic, curvilinear elastic: every quantity
}

}  // namespace

// Algorithmic bytes (inputs once, outputs once) and flops of one element of a class.
void class_cost(const stp_class& c, int io_bytes, double* bytes, double* flops)
{
    const double n = c.order + 1, n3 = n * n * n, n2 = n * n, m = c.nquant, N = c.order;
    const bool hasA = c.physics == STP_GENERIC && (c.flags & STP_A_PRESENT);
    const bool src = (c.flags & STP_SRC_POINT) != 0;
    double in = n3 * m;
    if (c.physics != STP_GENERIC) {
        const double np = param_count(c.physics);
        in += (c.flags & STP_PARAM_PER_ELEMENT) ? np : n3 * np;
    } else {
        const double per = (c.flags & STP_COEF_PER_ELEMENT) ? 3 * m * m : 3 * n3 * m * m;
        in += per * (hasA ? 2 : 1);
    }
    if (src) in += n3 + m + N;
    double out = n3 * m + ((c.flags & STP_FAVG_SUM) ? 1 : 3) * n3 * m + 6 * n2 * m * (hasA ? 2 : 1);
    if (bytes) *bytes = (in + out) * io_bytes;
    if (flops) {
        double contr = 0, point = 0;
        for (int d = 0; d < 3; ++d) {
            contr += 2.0 * n * n3 * quantities_read(c, d);
            if (c.physics == STP_ACOUSTIC) point += 2.0 * 2 * n3;
            else if (c.physics == STP_ELASTIC) point += 2.0 * 8 * n3;
            else if (c.physics == STP_ELASTIC_CURV) point += 2.0 * 24 * n3;  // the 24 nonzeros of B_d
            else point += 2.0 * m * m * n3;
            if (hasA) {
                contr += 2.0 * n * n3 * m;
                point += 2.0 * m * m * n3;
            }
        }
        double f = (N + 1) * (contr + point);  // N Taylor applications + the favg application
        f += 2.0 * n3 * m * N;                 // time accumulation
        f += 12.0 * n3 * m;                    // face extrapolation of q-bar
        if (hasA) f += 12.0 * n3 * m + 3 * 2.0 * m * m * n3;
        if (src) f += 3.0 * n3 * m * N;
        *flops = f;
    }
}

}  // namespace stp

using namespace stp;

namespace {

stp_status validate_class(const stp_class& c)
{
    if (c.order < 1 || c.order > kMaxOrder)
        return fail(STP_E_UNSUPPORTED, "order N=%d outside 1..%d", c.order, kMaxOrder);
    if (c.physics == STP_ACOUSTIC) {
        if (c.nquant != 4) return fail(STP_E_UNSUPPORTED, "acoustic preset needs m=4 (got %d)", c.nquant);
    } else if (c.physics == STP_ELASTIC || c.physics == STP_ELASTIC_CURV) {
        if (c.nquant != 9) return fail(STP_E_UNSUPPORTED, "elastic preset needs m=9 (got %d)", c.nquant);
    } else if (c.physics == STP_GENERIC) {
        if (c.nquant < 1 || c.nquant > 16)
            return fail(STP_E_UNSUPPORTED, "generic m=%d outside 1..16", c.nquant);
    } else {
        return fail(STP_E_INVAL, "unknown physics %d", c.physics);
    }
    const unsigned known = STP_PARAM_PER_ELEMENT | STP_A_PRESENT | STP_COEF_PER_ELEMENT | STP_FAVG_SUM | STP_SRC_POINT;
    if (c.flags & ~known) return fail(STP_E_INVAL, "unknown class flags 0x%x", c.flags & ~known);
    if (c.physics != STP_GENERIC && (c.flags & (STP_A_PRESENT | STP_COEF_PER_ELEMENT)))
        return fail(STP_E_INVAL, "A_PRESENT / COEF_PER_ELEMENT are generic-only flags");
    if (c.physics == STP_GENERIC && (c.flags & STP_PARAM_PER_ELEMENT))
        return fail(STP_E_INVAL, "PARAM_PER_ELEMENT is a preset-only flag");
    return STP_OK;
}

template <typename T>
stp_status upload(const T* host, size_t count, void** dev)
{
    hipError_t e = hipMalloc(dev, sizeof(T) * count);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(table)");
    e = hipMemcpy(*dev, host, sizeof(T) * count, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(table)");
    return STP_OK;
}

stp_status build_class(stp_plan_s* p, ClassState& cs)
{
    const int n = cs.cls.order + 1;
    double xi[kMaxNodes], w[kMaxNodes], D[kMaxNodes * kMaxNodes], e0[kMaxNodes], e1[kMaxNodes];
    if (p->nodes == 1)
        gauss_lobatto_01(n, xi, w);
    else
        gauss_legendre_01(n, xi, w);
    derivative_matrix(n, xi, D);
    lagrange_values(n, xi, 0.0, e0);
    lagrange_values(n, xi, 1.0, e1);
    stp_status st;
    if (p->prec == STP_FP64) {
        if ((st = upload(D, n * n, &cs.dD)) != STP_OK) return st;
        if ((st = upload(e0, n, &cs.de0)) != STP_OK) return st;
        if ((st = upload(e1, n, &cs.de1)) != STP_OK) return st;
        if ((st = upload(w, n, &cs.dw)) != STP_OK) return st;
    } else {
        float Df[kMaxNodes * kMaxNodes], e0f[kMaxNodes], e1f[kMaxNodes];
        derivative_matrix_f32(n, D, Df);
        for (int i = 0; i < n; ++i) {
            e0f[i] = (float)e0[i];
            e1f[i] = (float)e1[i];
        }
        if ((st = upload(Df, n * n, &cs.dD)) != STP_OK) return st;
        if ((st = upload(e0f, n, &cs.de0)) != STP_OK) return st;
        if ((st = upload(e1f, n, &cs.de1)) != STP_OK) return st;
        float wf[kMaxNodes];
        for (int i = 0; i < n; ++i) wf[i] = (float)w[i];
        if ((st = upload(wf, n, &cs.dw)) != STP_OK) return st;
        // FP64 face vectors for classes that accumulate in FP64
        if ((st = upload(e0, n, &cs.de0_64)) != STP_OK) return st;
        if ((st = upload(e1, n, &cs.de1_64)) != STP_OK) return st;
    }
    cs.acc64 = p->prec != STP_FP64 && p->acc64_min_order > 0 && cs.cls.order >= p->acc64_min_order;
    const bool hasA = cs.cls.physics == STP_GENERIC && (cs.cls.flags & STP_A_PRESENT);
    const KernelInfo chosen = select_kernel(p, cs, &cs.variant);
    if (!chosen.fn) return fail(STP_E_UNSUPPORTED, "no kernel for N=%d m=%d physics=%d", cs.cls.order,
                                cs.cls.nquant, cs.cls.physics);
    cs.cands = p->variant == STP_VARIANT_AUTO ? kernel_candidates(p, cs)
                                              : std::vector<std::pair<int, KernelInfo>>{{cs.variant, chosen}};
    bool needEvenOdd = false, needSplit = false;  // tables of every candidate (the tuner may switch)
    for (auto& c : cs.cands) {
        needEvenOdd |= c.second.aux == KernelInfo::kAuxEvenOdd;
        needSplit |= c.second.aux == KernelInfo::kAuxMfmaSplit;
    }
    if (needEvenOdd) {
        // even/odd split of D on the symmetric nodes: A = (D[i][j] - D[i][n-1-j])/2, B = (D[i][j] + D[i][n-1-j])/2
        // (i, j < n/2), Cm[i] = D[i][mid], Am[j] = D[mid][j] for odd n
        const int hh = n / 2;
        double t[2 * 5 * 5 + 2 * 5] = {0};
        for (int i = 0; i < hh; ++i)
            for (int j = 0; j < hh; ++j) {
                t[i * hh + j] = 0.5 * (D[i * n + j] - D[i * n + (n - 1 - j)]);
                t[hh * hh + i * hh + j] = 0.5 * (D[i * n + j] + D[i * n + (n - 1 - j)]);
            }
        if (n % 2)
            for (int i = 0; i < hh; ++i) {
                t[2 * hh * hh + i] = D[i * n + hh];
                t[2 * hh * hh + hh + i] = D[hh * n + i];
            }
        const int cnt = 2 * hh * hh + 2 * hh;
        if (p->prec == STP_FP64) {
            if ((st = upload(t, cnt > 0 ? cnt : 1, &cs.daux)) != STP_OK) return st;
        } else {
            float tf[2 * 5 * 5 + 2 * 5];
            for (int i = 0; i < cnt; ++i) tf[i] = (float)t[i];
            if ((st = upload(tf, cnt > 0 ? cnt : 1, &cs.daux)) != STP_OK) return st;
        }
    }
    if (needSplit) {
        // A operands of the MFMA kernels: D (the FP32 matrix with zero row sums) split exactly into three BF16
        // pieces D = D0 + D1 + D2, placed as each kernel's products expect (mfma_tables.cpp)
        float Df[kMaxNodes * kMaxNodes];
        derivative_matrix_f32(n, D, Df);
        uint16_t P0[kMaxNodes * kMaxNodes], P1[kMaxNodes * kMaxNodes], P2[kMaxNodes * kMaxNodes];
        split3_bf16(n * n, Df, P0, P1, P2);
        const std::vector<uint16_t> tab = n == 8 ? mfma_table_n8(P0, P1, P2) : mfma_table_hi(n, P0, P1, P2);
        if (tab.empty()) return fail(STP_E_DEVICE, "MFMA table for n=%d failed its consistency check", n);
        if ((st = upload(tab.data(), tab.size(), &cs.dDsplit)) != STP_OK) return st;
    }
    (void)hasA;
    if ((st = set_kernel(p, cs, chosen)) != STP_OK) return st;
    const int io = p->prec == STP_FP64 ? 8 : 4;
    class_cost(cs.cls, io, &cs.bytes, &cs.flops);
    const int64_t n3 = (int64_t)n * n * n, n2 = (int64_t)n * n, m = cs.cls.nquant;
    cs.size_q = n3 * m;
    cs.size_face = 6 * n2 * m;
    cs.size_src = n3 + m + cs.cls.order;
    if (cs.cls.physics == STP_GENERIC)
        cs.size_coef = (cs.cls.flags & STP_COEF_PER_ELEMENT) ? 3 * m * m : 3 * n3 * m * m;
    else
        cs.size_coef = (cs.cls.flags & STP_PARAM_PER_ELEMENT) ? param_count(cs.cls.physics)
                                                               : n3 * param_count(cs.cls.physics);
    return STP_OK;
}

void free_plan_memory(stp_plan_s* p)
{
    for (auto& cs : p->classes) {
        for (void* q : {cs.dD, cs.de0, cs.de1, cs.de0_64, cs.de1_64, cs.dDsplit, cs.daux, cs.dw})
            if (q) (void)hipFree(q);
    }
    for (void* q : {p->d_hcls, (void*)p->d_slots, (void*)p->d_orders, (void*)p->d_bncls, (void*)p->d_bad})
        if (q) (void)hipFree(q);
    free_scratch(p->run_scratch);
}

}  // namespace

extern "C" {

const char* stp_last_error(void) { return g_last_error.c_str(); }

stp_status stp_plan(const stp_plan_desc* desc, stp_plan_t* out)
{
    g_last_error.clear();
    if (!out) return fail(STP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!desc) return fail(STP_E_INVAL, "desc is NULL");
    if (desc->nclass < 1 || desc->nclass > kMaxClasses || !desc->classes)
        return fail(STP_E_INVAL, "nclass=%d outside 1..%d or classes NULL", desc->nclass, kMaxClasses);
    if (desc->prec < STP_FP64 || desc->prec > STP_BF16X3) return fail(STP_E_INVAL, "unknown precision %d", desc->prec);
    if (desc->acc64_min_order < 0) return fail(STP_E_INVAL, "acc64_min_order < 0");
    if (desc->variant < STP_VARIANT_AUTO || desc->variant > STP_VARIANT_MFMA)
        return fail(STP_E_INVAL, "unknown variant %d", desc->variant);
    if (desc->autotune < 0 || desc->autotune > 2) return fail(STP_E_INVAL, "autotune=%d outside 0..2", desc->autotune);
    if (desc->nodes < 0 || desc->nodes > 1) return fail(STP_E_INVAL, "nodes=%d outside 0..1", desc->nodes);
    for (int i = 0; i < desc->nclass; ++i) {
        stp_status st = validate_class(desc->classes[i]);
        if (st != STP_OK) return st;
    }
    if (desc->device < 0) return fail(STP_E_INVAL, "device %d < 0", desc->device);
    stp_status st0;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (desc->device >= ndev) return fail(STP_E_INVAL, "device %d of %d", desc->device, ndev);
    DeviceGuard g(desc->device);
    if ((st0 = static_scratch_init(desc->device)) != STP_OK) return st0;
    stp_plan_s* p = new (std::nothrow) stp_plan_s();
    if (!p) return fail(STP_E_NOMEM, "out of host memory");
    p->device = desc->device;
    p->prec = desc->prec;
    p->acc64_min_order = desc->acc64_min_order;
    p->variant = desc->variant;
    p->serve_budget = desc->serve_mem_budget;
    p->nodes = desc->nodes;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, desc->device)) != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    p->num_cus = prop.multiProcessorCount;
    p->classes.resize(desc->nclass);
    for (int i = 0; i < desc->nclass; ++i) {
        p->classes[i].cls = desc->classes[i];
        stp_status st = build_class(p, p->classes[i]);
        if (st != STP_OK) {
            free_plan_memory(p);
            delete p;
            return st;
        }
    }
    if (desc->nclass > 1) {
        stp_status st = hetero_prepare(p);
        if (st != STP_OK) {
            free_plan_memory(p);
            delete p;
            return st;
        }
    }
    p->autotune = desc->autotune;
    {
        stp_status st = autotune_plan(p, desc->autotune);
        if (st != STP_OK) {
            free_plan_memory(p);
            delete p;
            return st;
        }
    }
    if (p->serve_budget > 0) {
        stp_status st = serve_start(p);
        if (st != STP_OK) {
            free_plan_memory(p);
            delete p;
            return st;
        }
    }
    *out = p;
    return STP_OK;
}

void stp_plan_free(stp_plan_t p)
{
    if (!p) return;
    DeviceGuard g(p->device);
    serve_stop(p);
    (void)hipDeviceSynchronize();
    free_plan_memory(p);
    delete p;
}

stp_status stp_reserve(stp_plan_t p, int64_t max_nelem)
{
    g_last_error.clear();
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    if (max_nelem < 0 || max_nelem > (int64_t)INT32_MAX) return fail(STP_E_INVAL, "max_nelem out of range");
    if (p->classes.size() == 1) return STP_OK;  // uniform batches need no scratch
    DeviceGuard g(p->device);
    std::lock_guard<std::mutex> lk(p->run_mu);
    return reserve_scratch(p, p->run_scratch, max_nelem);
}

stp_status stp_plan_describe(stp_plan_t p, char* buf, size_t len)
{
    g_last_error.clear();
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    if (!buf || len == 0) return fail(STP_E_INVAL, "buffer is NULL or empty");
    static const char* names[] = {"auto", "plain", "fused", "mfma"};
    std::string out = "{\"classes\": [";
    char tmp[256];
    for (size_t c = 0; c < p->classes.size(); ++c) {
        const ClassState& cs = p->classes[c];
        const KernelInfo onchip = resident_kernel_f32(cs.cls.order, cs.cls.nquant);
        std::snprintf(tmp, sizeof tmp,
                      "%s{\"order\": %d, \"nquant\": %d, \"physics\": %d, \"variant\": \"%s\", \"tiled\": %s, "
                      "\"elements_per_tile\": %d, \"acc64\": %s, \"on_chip_B\": %s}",
                      c ? ", " : "", cs.cls.order, cs.cls.nquant, cs.cls.physics,
                      names[cs.variant >= 0 && cs.variant <= 3 ? cs.variant : 0], cs.tiled ? "true" : "false",
                      cs.tiled ? cs.slots : 1, cs.acc64 ? "true" : "false",
                      onchip.fn && onchip.fn == cs.kernel.fn ? "true" : "false");
        out += tmp;
    }
    std::snprintf(tmp, sizeof tmp,
                  "], \"hetero_grid_per_cu\": %d, \"hetero_lds_budget\": %zu, \"autotune\": %d, \"nodes\": \"%s\"}",
                  p->hetero_grid_per_cu, p->hetero_lds_budget, p->autotune, p->nodes ? "lobatto" : "legendre");
    out += tmp;
    if (out.size() + 1 > len) return fail(STP_E_INVAL, "buffer of %zu bytes too small (%zu needed)", len, out.size() + 1);
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return STP_OK;
}

stp_status stp_class_cost(stp_plan_t p, int cls, double* bytes, double* flops)
{
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    if (cls < 0 || cls >= (int)p->classes.size()) return fail(STP_E_INVAL, "class %d out of range", cls);
    if (bytes) *bytes = p->classes[cls].bytes;
    if (flops) *flops = p->classes[cls].flops;
    return STP_OK;
}

stp_status stp_run(stp_plan_t p, const stp_batch* b, void* stream)
{
    g_last_error.clear();
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    stp_status st = validate_batch(p, b);
    if (st != STP_OK) return st;
    if (b->nelem == 0) return STP_OK;
    DeviceGuard g(p->device);
    return launch_batch(p, b, static_cast<hipStream_t>(stream));
}

stp_status stp_sync(stp_plan_t p, void* stream)
{
    g_last_error.clear();
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    DeviceGuard g(p->device);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (!p->d_bad) return STP_OK;  // single-class plans have no class ids
    int32_t bad = 0;
    if ((e = hipMemcpy(&bad, p->d_bad, sizeof bad, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "hipMemcpy(flag)");
    if (!bad) return STP_OK;
    const int32_t zero = 0;
    if ((e = hipMemcpy(p->d_bad, &zero, sizeof zero, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy(flag)");
    return fail(STP_E_INVAL, "a batch run since the last stp_sync had class ids outside 0..%d; those elements' outputs "
                "were not written", (int)p->classes.size() - 1);
}

}  // extern "C"

namespace stp {

stp_status set_kernel(stp_plan_s* p, ClassState& cs, const KernelInfo& k)
{
    (void)p;
    const bool hasA = cs.cls.physics == STP_GENERIC && (cs.cls.flags & STP_A_PRESENT);
    const size_t lds = k.lds(cs.cls.nquant, hasA);
    if (lds > kMaxLds)
        return fail(STP_E_UNSUPPORTED, "class N=%d m=%d needs %zu B of LDS (> %zu)", cs.cls.order, cs.cls.nquant, lds,
                    (size_t)kMaxLds);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(LDS)");
    }
    cs.kernel = k;
    cs.lds = lds;
    for (auto& c : cs.cands)
        if (c.second.fn == k.fn) cs.variant = c.first;
    return STP_OK;
}

stp_status validate_batch(stp_plan_s* p, const stp_batch* b)
{
    if (!b) return fail(STP_E_INVAL, "batch is NULL");
    if (b->nelem < 0) return fail(STP_E_INVAL, "nelem < 0");
    if (b->nelem > (int64_t)INT32_MAX) return fail(STP_E_INVAL, "nelem > 2^31-1");
    if (b->nelem == 0) return STP_OK;
    const bool multi = p->classes.size() > 1;
    if (multi && (!b->cls || !b->off_q || !b->off_coef || !b->off_face))
        return fail(STP_E_INVAL, "heterogeneous plans need cls, off_q, off_coef and off_face");
    if (!b->dt || !b->h) return fail(STP_E_INVAL, "dt / h are NULL");
    if (b->dt_h_scalar) {
        if (!(b->h[0] > 0) || !std::isfinite(b->h[0])) return fail(STP_E_INVAL, "h must be > 0 (got %g)", b->h[0]);
        if (!(b->dt[0] >= 0) || !std::isfinite(b->dt[0])) return fail(STP_E_INVAL, "dt must be >= 0 (got %g)", b->dt[0]);
    }
    if (!b->Q || !b->qavg || !b->favg || !b->qface) return fail(STP_E_INVAL, "Q / qavg / favg / qface is NULL");
    bool anyA = false, anyPreset = false, anyGeneric = false, anySrc = false;
    for (auto& cs : p->classes) {
        anyA |= cs.cls.physics == STP_GENERIC && (cs.cls.flags & STP_A_PRESENT);
        anyPreset |= cs.cls.physics != STP_GENERIC;
        anyGeneric |= cs.cls.physics == STP_GENERIC;
        anySrc |= (cs.cls.flags & STP_SRC_POINT) != 0;
    }
    if (anyPreset && !b->params) return fail(STP_E_INVAL, "params is NULL for a preset class");
    if (anyGeneric && !b->B) return fail(STP_E_INVAL, "B is NULL for a generic class");
    if (anyA && (!b->A || !b->fface)) return fail(STP_E_INVAL, "A / fface is NULL for a class with A present");
    if (anySrc && !b->src) return fail(STP_E_INVAL, "src is NULL for a class with a point source");
    if (anySrc && multi && !b->off_src) return fail(STP_E_INVAL, "heterogeneous point sources need off_src");
    // outputs must not alias inputs or each other (checked on the element ranges of a uniform batch)
    if (!multi) {
        const ClassState& cs = p->classes[0];
        const int64_t io = p->prec == STP_FP64 ? 8 : 4, E = b->nelem;
        const int64_t fmul = (cs.cls.flags & STP_FAVG_SUM) ? 1 : 3;
        struct R { const void* p; int64_t bytes; const char* name; };
        std::vector<R> ins = {{b->Q, E * cs.size_q * io, "Q"}};
        if (b->params && cs.cls.physics != STP_GENERIC) ins.push_back({b->params, E * cs.size_coef * io, "params"});
        if (b->B && cs.cls.physics == STP_GENERIC) ins.push_back({b->B, E * cs.size_coef * io, "B"});
        if (b->A && anyA) ins.push_back({b->A, E * cs.size_coef * io, "A"});
        if (b->src && anySrc) ins.push_back({b->src, E * cs.size_src * io, "src"});
        std::vector<R> outs = {{b->qavg, E * cs.size_q * io, "qavg"}, {b->favg, E * fmul * cs.size_q * io, "favg"},
                               {b->qface, E * cs.size_face * io, "qface"}};
        if (anyA) outs.push_back({b->fface, E * cs.size_face * io, "fface"});
        auto overlap = [](const R& a, const R& c) {
            auto a0 = (uintptr_t)a.p, c0 = (uintptr_t)c.p;
            return a0 < c0 + (uintptr_t)c.bytes && c0 < a0 + (uintptr_t)a.bytes;
        };
        for (size_t i = 0; i < outs.size(); ++i) {
            for (auto& in : ins)
                if (overlap(outs[i], in)) return fail(STP_E_INVAL, "output %s aliases input %s", outs[i].name, in.name);
            for (size_t j = i + 1; j < outs.size(); ++j)
                if (overlap(outs[i], outs[j]))
                    return fail(STP_E_INVAL, "outputs %s and %s overlap", outs[i].name, outs[j].name);
        }
    }
    return STP_OK;
}

}  // namespace stp
