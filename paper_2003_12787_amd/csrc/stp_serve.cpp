// stp_serve.cpp -- serving runtime behind stp_submit / stp_poll / stp_drain.
//
// A plan created with serve_mem_budget > 0 owns kLanes serving lanes (a HIP stream at default priority, its
// own heterogeneous scratch and a completion thread each) and one dispatcher thread:
//   dispatcher : takes submitted batches in arrival order and admits one when the bytes of its outputs
//                plus heterogeneous scratch fit the budget next to the batches still in flight; it queues the
//                launches on the lane with the fewest batches in flight and records a completion event;
//   completers : one per lane, wait for that lane's events in launch order (one stream, so they finish in
//                order), stamp the completion time and release the batch's bytes.
// Completion events are pooled per lane. Heterogeneous batches report class ids outside the plan through a
// ring of pinned host words per lane, one per batch in flight: the bucketing pass writes the batch's word,
// and its completer turns it into the ticket's status.
// With STP_SERVE_SPLIT = k > 0, a batch larger than k elements is queued as parts of at most k elements
// (contiguous element ranges), which the dispatcher spreads over the lanes; its ticket completes when every
// part has. A ticket may carry a deadline: parts still queued when it passes are dropped and the ticket fails
// with STP_E_TIMEOUT.
// Small batches cannot fill the GPU and a batch takes at least as long as its slowest element, so several
// lanes let independent batches overlap. Tickets carry host monotonic timestamps (submit, launch, completion)
// for latency statistics.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "stp_plan.hpp"

namespace stp {

double now_seconds()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

namespace {

constexpr int kLanes = 4;
constexpr int kRing = 4096;  // flag words per lane: bounds the batches in flight on a lane
// Largest part of a batch on one lane; 0 = batches are not split. Splitting at 1024 elements lowered the
// saturated rate of the serving workload by 10% (each part repeats the bucketing pass and the class launches)
// and did not lower p99 at 80% load, so it is off unless STP_SERVE_SPLIT names a part size.
constexpr int64_t kSplitDefault = 0;

struct Pending {
    uint64_t ticket;
    stp_batch batch;
    double dt_s, h_s;  // copies of host scalars (the batch points at them when dt_h_scalar)
    size_t bytes;
    double deadline;   // latest launch time (host monotonic seconds); +inf without a timeout
};

struct InFlight {
    uint64_t ticket;
    hipEvent_t ev;
    size_t bytes;
    int slot;  // flag word of the batch in the lane's ring (-1: single-class plan)
};

struct TicketRec {
    stp_ticket_info info;
    int parts_left = 0;  // parts queued or in flight
};

struct Lane {
    hipStream_t stream = nullptr;
    HeteroScratch scratch;
    std::deque<InFlight> inflight;
    std::vector<hipEvent_t> events;   // completion events not in use
    int32_t* ring = nullptr;          // [kRing] pinned host flags (heterogeneous plans)
    int32_t* dring = nullptr;         // the same words as the device addresses them
    uint64_t seq = 0;                 // batches launched on the lane
    std::condition_variable cv;
    std::thread completer;
};

}  // namespace

struct ServeState {
    Lane lanes[kLanes];
    std::mutex mu;
    std::condition_variable cv_dispatch, cv_idle;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, TicketRec> tickets;
    size_t inflight_bytes = 0;
    int inflight_count = 0;
    int launching = 0;  // batches popped by the dispatcher whose launch is being queued
    uint64_t next_ticket = 1;
    int64_t split = kSplitDefault;  // batches above this many elements are queued as parts (0: never)
    bool stop = false;
    std::thread dispatcher;

    bool idle() const { return queue.empty() && inflight_count == 0 && launching == 0; }
};

namespace {

constexpr size_t kMaxPending = 65536;

size_t batch_bytes(const stp_plan_s* p, const stp_batch* b)
{
    const size_t io = p->prec == STP_FP64 ? 8 : 4;
    size_t per = 0;
    for (auto& cs : p->classes) {
        const bool hasA = cs.cls.physics == STP_GENERIC && (cs.cls.flags & STP_A_PRESENT);
        const size_t fmul = (cs.cls.flags & STP_FAVG_SUM) ? 1 : 3;
        size_t out = io * (cs.size_q * (1 + fmul) + cs.size_face * (hasA ? 2 : 1));
        per = std::max(per, out);
    }
    size_t scratch = p->classes.size() > 1 ? sizeof(int32_t) * p->classes.size() : 0;
    return (size_t)b->nelem * (per + scratch);
}

// The lane with the fewest batches in flight. (Choosing by in-flight bytes instead measured the same.)
int least_loaded(const ServeState* s)
{
    int li = 0;
    for (int l = 1; l < kLanes; ++l)
        if (s->lanes[l].inflight.size() < s->lanes[li].inflight.size()) li = l;
    return li;
}

// Elements [a, a + k) of batch b as a batch of their own: per-element arrays advance by a; contiguous data
// (NULL offset arrays) advance by a elements of the single class.
stp_batch part_of(const stp_plan_s* p, const stp_batch& b, int64_t a, int64_t k)
{
    stp_batch s = b;
    s.nelem = k;
    const int64_t io = p->prec == STP_FP64 ? 8 : 4;
    const ClassState& cs = p->classes[0];
    auto adv = [&](const void* ptr, int64_t values) -> const void* {
        return ptr ? static_cast<const char*>(ptr) + a * values * io : nullptr;
    };
    auto advm = [&](void* ptr, int64_t values) -> void* {
        return ptr ? static_cast<char*>(ptr) + a * values * io : nullptr;
    };
    if (b.cls) s.cls = b.cls + a;
    if (b.off_q) {
        s.off_q = b.off_q + a;
    } else {
        const int64_t fmul = (cs.cls.flags & STP_FAVG_SUM) ? 1 : 3;
        s.Q = adv(b.Q, cs.size_q);
        s.qavg = advm(b.qavg, cs.size_q);
        s.favg = advm(b.favg, fmul * cs.size_q);
    }
    if (b.off_coef) {
        s.off_coef = b.off_coef + a;
    } else {
        s.params = adv(b.params, cs.size_coef);
        s.A = adv(b.A, cs.size_coef);
        s.B = adv(b.B, cs.size_coef);
    }
    if (b.off_face) {
        s.off_face = b.off_face + a;
    } else {
        s.qface = advm(b.qface, cs.size_face);
        s.fface = advm(b.fface, cs.size_face);
    }
    if (b.off_src) s.off_src = b.off_src + a;
    else s.src = adv(b.src, cs.size_src);
    if (!b.dt_h_scalar) {
        s.dt = b.dt + a;
        s.h = b.h + a;
    }
    return s;
}

// One part of a ticket has ended with status st: the ticket completes when its last part has, with the first
// failure of its parts.
void part_done(ServeState* s, uint64_t ticket, stp_status st, double t)
{
    auto& r = s->tickets[ticket];
    if (st != STP_OK && (r.info.status == STP_PENDING || r.info.status == STP_OK)) r.info.status = st;
    r.info.t_done = std::max(r.info.t_done, t);
    if (--r.parts_left == 0 && r.info.status == STP_PENDING) r.info.status = STP_OK;
}

void dispatcher_main(stp_plan_s* p)
{
    ServeState* s = p->serve;
    (void)hipSetDevice(p->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        auto ready = [&] {
            return (!s->queue.empty() && ((s->inflight_bytes + s->queue.front().bytes <= p->serve_budget &&
                                           s->lanes[least_loaded(s)].inflight.size() < (size_t)kRing) ||
                                          now_seconds() >= s->queue.front().deadline)) ||
                   (s->stop && s->queue.empty());
        };
        while (!ready()) {
            // wake for a completion, a submission, or the deadline of the batch at the front
            if (!s->queue.empty() && s->queue.front().deadline < 1e300) {
                const auto wait = std::chrono::duration<double>(
                    std::max(0.0, s->queue.front().deadline - now_seconds()) + 1e-4);
                s->cv_dispatch.wait_for(lk, wait);
            } else {
                s->cv_dispatch.wait(lk);
            }
        }
        if (s->queue.empty()) break;  // stopping, nothing left to launch
        Pending job = s->queue.front();
        s->queue.pop_front();
        if (now_seconds() >= job.deadline) {  // too late to start: dropped, the ticket fails
            part_done(s, job.ticket, STP_E_TIMEOUT, now_seconds());
            if (s->idle()) s->cv_idle.notify_all();
            continue;
        }
        s->inflight_bytes += job.bytes;
        ++s->launching;
        Lane& lane = s->lanes[least_loaded(s)];
        {
            auto& info = s->tickets[job.ticket].info;
            if (info.t_start == 0) info.t_start = now_seconds();
        }
        hipEvent_t ev = nullptr;
        if (!lane.events.empty()) {
            ev = lane.events.back();
            lane.events.pop_back();
        }
        lk.unlock();
        if (job.batch.dt_h_scalar) {
            job.batch.dt = &job.dt_s;
            job.batch.h = &job.h_s;
        }
        int slot = -1;
        if (lane.ring) {  // the batch's flag word; its previous batch has completed (at most kRing in flight)
            slot = (int)(lane.seq++ % kRing);
            lane.ring[slot] = 0;
            lane.scratch.bad = lane.dring + slot;
        }
        // Only this thread launches on a lane, so its scratch is not shared by overlapping launches.
        stp_status st = launch_batch(p, &job.batch, lane.stream, &lane.scratch);
        if (st == STP_OK) {
            hipError_t e = ev ? hipSuccess : hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventRecord(ev, lane.stream);
            if (e != hipSuccess) st = STP_E_DEVICE;
        }
        lk.lock();
        --s->launching;
        if (st != STP_OK) {
            if (ev) lane.events.push_back(ev);
            part_done(s, job.ticket, st, now_seconds());
            s->inflight_bytes -= job.bytes;
            if (s->idle()) s->cv_idle.notify_all();
            continue;
        }
        lane.inflight.push_back({job.ticket, ev, job.bytes, slot});
        ++s->inflight_count;
        lane.cv.notify_one();
    }
    for (auto& l : s->lanes) l.cv.notify_all();
}

void completer_main(stp_plan_s* p, int li)
{
    ServeState* s = p->serve;
    Lane& lane = s->lanes[li];
    (void)hipSetDevice(p->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        lane.cv.wait(lk, [&] { return !lane.inflight.empty() || (s->stop && s->queue.empty() && s->launching == 0); });
        if (lane.inflight.empty()) break;  // stopping and everything of this lane has completed
        InFlight f = lane.inflight.front();
        lk.unlock();
        hipError_t e = hipEventSynchronize(f.ev);
        double t = now_seconds();
        const bool bad = f.slot >= 0 && reinterpret_cast<volatile int32_t*>(lane.ring)[f.slot] != 0;
        lk.lock();
        lane.events.push_back(f.ev);
        lane.inflight.pop_front();
        --s->inflight_count;
        part_done(s, f.ticket, e != hipSuccess ? STP_E_DEVICE : (bad ? STP_E_INVAL : STP_OK), t);
        s->inflight_bytes -= f.bytes;
        s->cv_dispatch.notify_one();
        if (s->idle()) s->cv_idle.notify_all();
    }
}

}  // namespace

stp_status serve_start(stp_plan_s* p)
{
    auto* s = new (std::nothrow) ServeState();
    if (!s) return fail(STP_E_NOMEM, "out of host memory");
    for (auto& l : s->lanes) {
        hipError_t e = hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (auto& m : s->lanes)
                if (m.stream) (void)hipStreamDestroy(m.stream);
            delete s;
            return hip_fail(e, "hipStreamCreate(serving)");
        }
    }
    if (p->classes.size() > 1) {
        // Heterogeneous scratch sized up front for the largest batch the budget admits (at most 64 Ki elements),
        // so that the dispatcher does not synchronise the device to grow it in the common case.
        stp_batch one{};
        one.nelem = 1;
        const int64_t cap = std::min<int64_t>(65536, std::max<int64_t>(1, (int64_t)(p->serve_budget / batch_bytes(p, &one))));
        for (auto& l : s->lanes) {
            stp_status st = reserve_scratch(p, l.scratch, cap);
            if (st == STP_OK) {
                hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&l.ring), sizeof(int32_t) * kRing, hipHostMallocMapped);
                if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&l.dring), l.ring, 0);
                if (e != hipSuccess) st = hip_fail(e, "hipHostMalloc(serving flags)");
                else std::memset(l.ring, 0, sizeof(int32_t) * kRing);
            }
            if (st != STP_OK) {
                for (auto& m : s->lanes) {
                    free_scratch(m.scratch);
                    if (m.ring) (void)hipHostFree(m.ring);
                    if (m.stream) (void)hipStreamDestroy(m.stream);
                }
                delete s;
                return st;
            }
        }
    }
    if (const char* e = std::getenv("STP_SERVE_SPLIT")) s->split = std::max<int64_t>(0, std::atoll(e));
    p->serve = s;
    s->dispatcher = std::thread(dispatcher_main, p);
    for (int l = 0; l < kLanes; ++l) s->lanes[l].completer = std::thread(completer_main, p, l);
    return STP_OK;
}

void serve_stop(stp_plan_s* p)
{
    ServeState* s = p->serve;
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_dispatch.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    for (auto& l : s->lanes) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            l.cv.notify_all();
        }
        if (l.completer.joinable()) l.completer.join();
    }
    for (auto& l : s->lanes) {
        (void)hipStreamSynchronize(l.stream);
        (void)hipStreamDestroy(l.stream);
        free_scratch(l.scratch);
        for (hipEvent_t ev : l.events) (void)hipEventDestroy(ev);
        if (l.ring) (void)hipHostFree(l.ring);
    }
    delete s;
    p->serve = nullptr;
}

}  // namespace stp

using namespace stp;

extern "C" {

stp_status stp_submit_deadline(stp_plan_t p, const stp_batch* b, double timeout_s, uint64_t* ticket)
{
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    if (!ticket) return fail(STP_E_INVAL, "ticket is NULL");
    if (!p->serve) return fail(STP_E_INVAL, "plan was created without a serving budget");
    if (!(timeout_s >= 0)) return fail(STP_E_INVAL, "timeout %g s is negative or NaN", timeout_s);
    stp_status st = validate_batch(p, b);
    if (st != STP_OK) return st;
    const int64_t split = p->serve->split;
    const int64_t nparts = split > 0 && b->nelem > split ? (b->nelem + split - 1) / split : 1;
    const int64_t per = b->nelem > 0 ? (b->nelem + nparts - 1) / nparts : 0;
    if (batch_bytes(p, b) > p->serve_budget * (size_t)nparts)  // every part must fit the budget on its own
        return fail(STP_E_NOMEM, "batch needs %zu B, more than the serving budget %zu B", batch_bytes(p, b),
                    p->serve_budget);
    ServeState* s = p->serve;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->queue.size() + (size_t)nparts > kMaxPending) return fail(STP_E_BUSY, "serving queue full");
    const double now = now_seconds();
    const uint64_t id = s->next_ticket++;
    TicketRec rec{};
    rec.info.t_submit = now;
    rec.info.status = STP_PENDING;
    std::vector<Pending> parts;
    for (int64_t a = 0; a < b->nelem; a += per) {
        Pending job{};
        job.ticket = id;
        job.batch = nparts > 1 ? part_of(p, *b, a, std::min(per, b->nelem - a)) : *b;
        job.bytes = batch_bytes(p, &job.batch);
        if (job.bytes > p->serve_budget)
            return fail(STP_E_NOMEM, "a part of %lld elements needs %zu B, more than the serving budget %zu B",
                        (long long)job.batch.nelem, job.bytes, p->serve_budget);
        job.deadline = timeout_s < 1e300 ? now + timeout_s : 1e308;
        if (b->dt_h_scalar) {
            job.dt_s = b->dt[0];
            job.h_s = b->h[0];
        }
        parts.push_back(job);
    }
    rec.parts_left = (int)parts.size();
    if (parts.empty()) {  // nothing to launch: complete immediately
        rec.info.t_start = rec.info.t_done = now;
        rec.info.status = STP_OK;
    }
    s->tickets[id] = rec;
    for (auto& job : parts) s->queue.push_back(job);
    if (!parts.empty()) s->cv_dispatch.notify_one();
    *ticket = id;
    return STP_OK;
}

stp_status stp_submit(stp_plan_t p, const stp_batch* b, uint64_t* ticket)
{
    return stp_submit_deadline(p, b, HUGE_VAL, ticket);
}

stp_status stp_poll(stp_plan_t p, uint64_t ticket, stp_ticket_info* info)
{
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    if (!p->serve) return fail(STP_E_INVAL, "plan was created without a serving budget");
    ServeState* s = p->serve;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return fail(STP_E_INVAL, "unknown or retired ticket %llu", (unsigned long long)ticket);
    if (info) *info = it->second.info;
    stp_status st = (stp_status)it->second.info.status;
    if (st == STP_PENDING) return STP_PENDING;
    s->tickets.erase(it);
    if (st == STP_E_INVAL)
        return fail(st, "ticket %llu had class ids outside 0..%d; those elements' outputs were not written",
                    (unsigned long long)ticket, (int)p->classes.size() - 1);
    if (st == STP_E_TIMEOUT)
        return fail(st, "ticket %llu: its deadline passed before all of its batch was launched; the elements "
                    "not launched were not written", (unsigned long long)ticket);
    if (st != STP_OK) return fail(st, "ticket %llu failed on the device", (unsigned long long)ticket);
    return STP_OK;
}

stp_status stp_drain(stp_plan_t p)
{
    if (!p) return fail(STP_E_INVAL, "plan is NULL");
    if (!p->serve) return STP_OK;
    ServeState* s = p->serve;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_idle.wait(lk, [&] { return s->idle(); });
    return STP_OK;
}

}  // extern "C"
