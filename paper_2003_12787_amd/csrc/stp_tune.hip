// stp_tune.hip -- plan-time autotuner with a JSON cache.
//
// What is tuned (plans created with variant = STP_VARIANT_AUTO):
//   * every class that runs as its own launch: the kernel variant (plain, fused, split-BF16 MFMA, whichever
//     exist for the class), timed on a synthetic batch of the class;
//   * heterogeneous plans: the persistent grid (workgroups per CU) and the LDS budget of a tile, which sets
//     the elements per workgroup of every tiled class; timed on a synthetic batch with equal counts per class.
// Results are cached in a JSON file (STP_TUNE_CACHE, else $HOME/.cache/stp_tune.json) under keys that name the
// architecture, the HIP runtime version and the class (order, quantity count, physics, flags, precision,
// FP64 accumulation). autotune = 0 uses cached entries and otherwise the built-in rules; 1 also tunes what
// the cache lacks and stores it; 2 retunes everything. Inputs of the timing batches are filled on the
// device with bounded values (positive material parameters), dt = 1e-3, h = 1.
#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "stp_plan.hpp"
#include "tune_cache.hpp"

namespace stp {

namespace {

// x[i] = lo + span * frac(i * golden): bounded, deterministic, no host traffic
template <typename T>
__global__ void fill_kernel(T* x, int64_t n, double lo, double span)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double f = (double)((uint64_t)(i * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
        x[i] = (T)(lo + span * f);
    }
}

// --------------------------------------------------------------------------------------------- JSON cache
// The cache is one JSON object: key -> object of numbers (tune_cache.cpp parses and formats it).
using Entry = TuneEntry;
using Cache = TuneCache;

std::string cache_path()
{
    if (const char* e = std::getenv("STP_TUNE_CACHE")) return e;
    const char* h = std::getenv("HOME");
    return std::string(h ? h : ".") + "/.cache/stp_tune.json";
}

Cache load_cache()
{
    Cache c;
    FILE* f = std::fopen(cache_path().c_str(), "rb");
    if (!f) return c;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
    std::fclose(f);
    (void)parse_tune_cache(s, c);  // a malformed cache reads as empty (only costs retuning)
    return c;
}

void store_cache(const Cache& c)
{
    const std::string path = cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        const std::string dir = path.substr(0, slash);
        for (size_t p = 1; p <= dir.size(); ++p)  // create missing levels (errors show up at fopen)
            if (p == dir.size() || dir[p] == '/') (void)mkdir(dir.substr(0, p).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;  // an unwritable cache only costs retuning
    const std::string text = format_tune_cache(c);
    std::fwrite(text.data(), 1, text.size(), f);
    std::fclose(f);
    (void)std::rename(tmp.c_str(), path.c_str());
}


// --------------------------------------------------------------------------------------------- keys
std::string device_tag(const stp_plan_s* p)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    int rt = 0;
    (void)hipRuntimeGetVersion(&rt);
    return arch + "|hip" + std::to_string(rt) + "|cu" + std::to_string(p->num_cus);
}

std::string class_key(const stp_plan_s* p, const ClassState& cs)
{
    std::ostringstream k;
    k << "N" << cs.cls.order << ",m" << cs.cls.nquant << ",p" << cs.cls.physics << ",f" << cs.cls.flags << ",prec"
      << p->prec << ",acc" << (cs.acc64 ? 1 : 0);
    return k.str();
}

// --------------------------------------------------------------------------------------------- probes
struct Probe {
    std::vector<void*> bufs;
    stp_batch b{};
    double dt = 1e-3, h = 1.0;
    ~Probe()
    {
        for (void* q : bufs) (void)hipFree(q);
    }
};

template <typename T>
stp_status alloc_fill(Probe& pr, int64_t n, double lo, double span, const void** out, hipStream_t st)
{
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(tuning batch)");
    pr.bufs.push_back(q);
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_kernel<T>, dim3(std::max(grid, 1)), dim3(256), 0, st, static_cast<T*>(q), n, lo, span);
    *out = q;
    return STP_OK;
}

// A synthetic batch with counts[c] elements of class c (element ids grouped by class, offsets given).
stp_status make_probe(stp_plan_s* p, const std::vector<int64_t>& counts, Probe& pr, hipStream_t st)
{
    const bool f64 = p->prec == STP_FP64;
    const int nclass = (int)p->classes.size();
    int64_t E = 0, nq = 0, nf = 0, npar = 0, ncoef = 0, nsrc = 0;
    bool anyA = false, anySrc = false, anyPreset = false, anyGen = false;
    std::vector<int32_t> cls;
    std::vector<int64_t> oq, oc, of, os;
    for (int c = 0; c < nclass; ++c) {
        const ClassState& cs = p->classes[c];
        const bool gen = cs.cls.physics == STP_GENERIC;
        for (int64_t k = 0; k < counts[c]; ++k) {
            cls.push_back(c);
            oq.push_back(nq);
            of.push_back(nf);
            os.push_back(nsrc);
            oc.push_back(gen ? ncoef : npar);
            nq += cs.size_q;
            nf += cs.size_face;
            (gen ? ncoef : npar) += cs.size_coef;
            if (cs.cls.flags & STP_SRC_POINT) nsrc += cs.size_src;
        }
        if (counts[c] > 0) {
            anyA |= gen && (cs.cls.flags & STP_A_PRESENT);
            anySrc |= (cs.cls.flags & STP_SRC_POINT) != 0;
            anyPreset |= !gen;
            anyGen |= gen;
        }
        E += counts[c];
    }
    pr.b.nelem = E;
    auto fill = [&](int64_t n, double lo, double span, const void** out) {
        return f64 ? alloc_fill<double>(pr, n, lo, span, out, st) : alloc_fill<float>(pr, n, lo, span, out, st);
    };
    stp_status s;
    if ((s = fill(nq, -0.5, 1.0, &pr.b.Q)) != STP_OK) return s;
    if (anyPreset && (s = fill(npar, 2.0, 1.0, &pr.b.params)) != STP_OK) return s;
    if (anyGen && (s = fill(ncoef, -0.2, 0.4, &pr.b.B)) != STP_OK) return s;
    if (anyA && (s = fill(ncoef, -0.2, 0.4, &pr.b.A)) != STP_OK) return s;
    if (anySrc && (s = fill(nsrc, 0.0, 1.0, &pr.b.src)) != STP_OK) return s;
    const void* o;
    if ((s = fill(nq, 0, 0, &o)) != STP_OK) return s;
    pr.b.qavg = const_cast<void*>(o);
    if ((s = fill(3 * nq, 0, 0, &o)) != STP_OK) return s;
    pr.b.favg = const_cast<void*>(o);
    if ((s = fill(nf, 0, 0, &o)) != STP_OK) return s;
    pr.b.qface = const_cast<void*>(o);
    if (anyA) {
        if ((s = fill(nf, 0, 0, &o)) != STP_OK) return s;
        pr.b.fface = const_cast<void*>(o);
    }
    pr.b.dt = &pr.dt;
    pr.b.h = &pr.h;
    pr.b.dt_h_scalar = 1;
    if (nclass > 1) {
        auto up = [&](const void* src, size_t bytes, const void** out) -> stp_status {
            void* q = nullptr;
            hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 8));
            if (e != hipSuccess) return hip_fail(e, "hipMalloc(tuning offsets)");
            pr.bufs.push_back(q);
            if (bytes && (e = hipMemcpy(q, src, bytes, hipMemcpyHostToDevice)) != hipSuccess)
                return hip_fail(e, "hipMemcpy(tuning offsets)");
            *out = q;
            return STP_OK;
        };
        const void* q;
        if ((s = up(cls.data(), cls.size() * 4, &q)) != STP_OK) return s;
        pr.b.cls = static_cast<const int32_t*>(q);
        if ((s = up(oq.data(), oq.size() * 8, &q)) != STP_OK) return s;
        pr.b.off_q = static_cast<const int64_t*>(q);
        if ((s = up(oc.data(), oc.size() * 8, &q)) != STP_OK) return s;
        pr.b.off_coef = static_cast<const int64_t*>(q);
        if ((s = up(of.data(), of.size() * 8, &q)) != STP_OK) return s;
        pr.b.off_face = static_cast<const int64_t*>(q);
        if ((s = up(os.data(), os.size() * 8, &q)) != STP_OK) return s;
        pr.b.off_src = static_cast<const int64_t*>(q);
    }
    hipError_t e = hipStreamSynchronize(st);
    return e == hipSuccess ? STP_OK : hip_fail(e, "hipStreamSynchronize(tuning batch)");
}

// Median of `reps` launches (after one warm-up), in milliseconds.
stp_status time_batch(stp_plan_s* p, const stp_batch* b, hipStream_t st, HeteroScratch* scr, double* ms)
{
    constexpr int reps = 5;
    hipEvent_t ev[reps + 1];
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(STP_E_DEVICE, "hipEventCreate");
    stp_status s = launch_batch(p, b, st, scr);
    for (int r = 0; r < reps && s == STP_OK; ++r) {
        (void)hipEventRecord(ev[r], st);
        s = launch_batch(p, b, st, scr);
    }
    (void)hipEventRecord(ev[reps], st);
    hipError_t e = hipEventSynchronize(ev[reps]);
    std::vector<float> t(reps);
    for (int r = 0; r < reps; ++r) (void)hipEventElapsedTime(&t[r], ev[r], ev[r + 1]);
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (s != STP_OK) return s;
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(tuning)");
    std::sort(t.begin(), t.end());
    *ms = t[reps / 2];
    return STP_OK;
}

constexpr double kProbeBytes = 512.0 * (1 << 20);  // inputs + outputs of a timing batch

}  // namespace

stp_status autotune_plan(stp_plan_s* p, int mode)
{
    if (p->variant != STP_VARIANT_AUTO) return STP_OK;
    Cache cache = load_cache();
    const std::string tag = device_tag(p);
    bool dirty = false;
    hipStream_t st = nullptr;
    auto stream = [&]() -> hipStream_t {
        if (!st) (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        return st;
    };
    stp_status s = STP_OK;
    const int nclass = (int)p->classes.size();
    // the kernel variant of a single-class plan (in heterogeneous plans every class with a choice of
    // variant is tiled: FP32 I/O, no FP64 accumulation, N <= 7)
    if (nclass == 1 && p->classes[0].cands.size() > 1) {
        ClassState& cs = p->classes[0];
        const std::string key = tag + "|class|" + class_key(p, cs);
        auto it = cache.find(key);
        if (it != cache.end() && mode < 2) {
            const int v = (int)it->second["variant"];
            for (auto& cand : cs.cands)
                if (cand.first == v) s = set_kernel(p, cs, cand.second);
        } else if (mode > 0) {
            const int64_t E = std::min<int64_t>(
                65536, std::max<int64_t>(p->num_cus, (int64_t)(kProbeBytes / std::max(cs.bytes, 1.0))));
            Probe pr;
            s = make_probe(p, {E}, pr, stream());
            double best = 1e30;
            int bestv = -1;
            KernelInfo bestk;
            for (auto& cand : cs.cands) {
                if (s != STP_OK) break;
                if ((s = set_kernel(p, cs, cand.second)) != STP_OK) break;
                double ms = 0;
                if ((s = time_batch(p, &pr.b, stream(), nullptr, &ms)) != STP_OK) break;
                if (ms < best) {
                    best = ms;
                    bestv = cand.first;
                    bestk = cand.second;
                }
            }
            if (s == STP_OK && bestv >= 0) {
                s = set_kernel(p, cs, bestk);
                cache[key] = Entry{{"variant", (double)bestv}, {"us_per_elem", best * 1e3 / (double)E}};
                dirty = true;
            }
        }
    }
    // heterogeneous plans: persistent grid and tile LDS budget
    if (s == STP_OK && nclass > 1) {
        std::ostringstream k;
        k << tag << "|hetero|prec" << p->prec;
        for (auto& cs : p->classes) k << ";" << class_key(p, cs);
        const std::string key = k.str();
        auto it = cache.find(key);
        if (it != cache.end() && mode < 2) {
            p->hetero_grid_per_cu = (int)it->second["grid_per_cu"];
            p->hetero_lds_budget = (size_t)it->second["lds_kb"] * 1024;
            s = hetero_prepare(p);
        } else if (mode > 0) {
            double per = 0;
            for (auto& cs : p->classes) per += cs.bytes;
            const int64_t each = std::max<int64_t>(8, std::min<int64_t>(4096, (int64_t)(kProbeBytes / per)));
            std::vector<int64_t> counts(nclass, each);
            Probe pr;
            HeteroScratch scr;
            s = make_probe(p, counts, pr, stream());
            if (s == STP_OK) s = reserve_scratch(p, scr, pr.b.nelem);
            double best = 1e30;
            int bg = p->hetero_grid_per_cu;
            size_t bl = p->hetero_lds_budget;
            for (int g : {2, 4, 8})
                for (size_t kb : {48, 80, 128}) {
                    if (s != STP_OK) break;
                    p->hetero_grid_per_cu = g;
                    p->hetero_lds_budget = kb * 1024;
                    if ((s = hetero_prepare(p)) != STP_OK) break;
                    double ms = 0;
                    if ((s = time_batch(p, &pr.b, stream(), &scr, &ms)) != STP_OK) break;
                    if (ms < best) {
                        best = ms;
                        bg = g;
                        bl = kb * 1024;
                    }
                }
            free_scratch(scr);
            if (s == STP_OK) {
                p->hetero_grid_per_cu = bg;
                p->hetero_lds_budget = bl;
                s = hetero_prepare(p);
                cache[key] = Entry{{"grid_per_cu", (double)bg}, {"lds_kb", (double)(bl / 1024)}, {"ms", best},
                                   {"elements", (double)pr.b.nelem}};
                dirty = true;
            }
        }
    }
    if (st) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (dirty && s == STP_OK) store_cache(cache);
    return s;
}

}  // namespace stp
