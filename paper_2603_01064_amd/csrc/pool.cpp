// Serving pool: continuous batching across several handles (typically one
// per grid size), with admission by a device-memory budget.
//
// Every right-hand side is an independent solve (Sec. 2.3), so requests of
// different sizes and alphas can be in flight together: each member handle
// runs its own slot engine on its own stream, and a pool step advances every
// member whose previous outer iteration has finished by one more (waiting
// for the first to finish when none has).  Members therefore iterate at
// their own pace: a small grid is not held to the iteration time of a large
// one, and the iterations of different members overlap on the device.
// Requests wait in one FIFO and enter their member's engine while the
// request bytes admitted so far (request_bytes of each request's handle)
// stay within the budget.

#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "nmg_internal.h"

struct nmg_pool_ctx {
    struct Member {
        nmg_handle h = nullptr;
        hipStream_t s = nullptr;
        hipEvent_t retired = nullptr;
        hipEvent_t iter_done = nullptr;  // recorded after each of the member's steps
        bool launched = false;           // iter_done has been recorded
    };
    struct Pending {
        long long id;
        int member;
        double alpha;
        int ws;
        const double* b;
        double* x;
        size_t bytes;
        double t_submit;
    };
    size_t budget = 0;
    size_t in_flight = 0;
    int precision = -1;  // cycle precision of the admitted requests
    std::vector<Member> members;
    std::deque<Pending> queue;
    std::unordered_map<long long, Pending> running;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

using nmg::fail;

extern "C" {

nmg_status nmg_pool_create(size_t hbm_budget_bytes, nmg_pool* out) {
    if (!out) return fail(NMG_ERR_ARG, "null argument");
    *out = nullptr;
    if (hbm_budget_bytes == 0) return fail(NMG_ERR_ARG, "the budget must be positive");
    auto* p = new nmg_pool_ctx();
    p->budget = hbm_budget_bytes;
    *out = p;
    return NMG_OK;
}

void nmg_pool_destroy(nmg_pool p) {
    if (!p) return;
    for (auto& m : p->members) {
        if (m.s) {
            (void)hipStreamSynchronize(m.s);
            (void)hipStreamDestroy(m.s);
        }
        if (m.retired) (void)hipEventDestroy(m.retired);
        if (m.iter_done) (void)hipEventDestroy(m.iter_done);
        (void)nmg_serve_reset(m.h);  // requests still in flight are abandoned
    }
    delete p;
}

nmg_status nmg_pool_add(nmg_pool p, nmg_handle h, int* member_out) {
    if (!p || !h || !member_out) return fail(NMG_ERR_ARG, "null argument");
    for (const auto& m : p->members)
        if (m.h == h) return fail(NMG_ERR_ARG, "handle already in the pool");
    if (!h->eng.queue.empty() || !h->eng.slot.empty())
        return fail(NMG_ERR_STATE, "the handle is serving requests of its own");
    nmg_pool_ctx::Member m;
    m.h = h;
    NMG_HIP(hipStreamCreateWithFlags(&m.s, hipStreamNonBlocking));
    NMG_HIP(hipEventCreateWithFlags(&m.retired, hipEventDisableTiming));
    NMG_HIP(hipEventCreateWithFlags(&m.iter_done, hipEventDisableTiming));
    p->members.push_back(m);
    *member_out = (int)p->members.size() - 1;
    return NMG_OK;
}

nmg_status nmg_pool_submit(nmg_pool p, int member, long long id, double alpha, int weight_set, const double* b_dev,
                           double* x_dev) {
    if (!p) return fail(NMG_ERR_ARG, "null pool");
    if (member < 0 || member >= (int)p->members.size()) return fail(NMG_ERR_ARG, "member out of range");
    if (!b_dev || !x_dev) return fail(NMG_ERR_ARG, "null pointer");
    nmg_handle h = p->members[(size_t)member].h;
    NMG_TRY(nmg::check_alpha(h, alpha, 0));
    if (weight_set < 0 || weight_set >= h->p.n_weight_sets) return fail(NMG_ERR_ARG, "weight set out of range");
    if (p->running.count(id)) return fail(NMG_ERR_ARG, "request id already in flight");
    for (const auto& q : p->queue)
        if (q.id == id) return fail(NMG_ERR_ARG, "request id already queued");
    // sized for mixed precision here; checked again against the step's precision
    const size_t bytes = nmg::request_bytes(h, NMG_MIXED);
    if (bytes > p->budget) return fail(NMG_ERR_ARG, "one request of this size exceeds the pool's budget");
    p->queue.push_back({id, member, alpha, weight_set, b_dev, x_dev, bytes, p->now_ms()});
    return NMG_OK;
}

nmg_status nmg_pool_step(nmg_pool p, double rtol, int max_cycles, const nmg_cycle_opts* o, nmg_request_result* done,
                         int* done_member, int capacity, int* n_done) {
    if (n_done) *n_done = 0;
    if (!p || !done || !done_member || !n_done) return fail(NMG_ERR_ARG, "null argument");
    if (!(rtol > 0.0) || max_cycles < 0) return fail(NMG_ERR_ARG, "rtol must be > 0 and max_cycles >= 0");
    for (const auto& m : p->members) NMG_TRY(nmg::check_opts(m.h, o));
    if (!p->running.empty() && p->precision != (int)o->precision)
        return fail(NMG_ERR_STATE, "cycle precision changed while requests are in flight");
    // ---- admission in arrival order while the budget allows (the head of
    // the queue is always admitted when nothing is in flight, so a request
    // larger than the budget at this precision cannot block the pool)
    while (!p->queue.empty()) {
        nmg_pool_ctx::Pending q = p->queue.front();
        q.bytes = nmg::request_bytes(p->members[(size_t)q.member].h, o->precision);
        if (p->in_flight + q.bytes > p->budget && !p->running.empty()) break;
        nmg_handle h = p->members[(size_t)q.member].h;
        NMG_TRY(nmg_serve_submit(h, q.id, q.alpha, q.ws, q.b, q.x));
        p->queue.pop_front();
        p->in_flight += q.bytes;
        p->running.emplace(q.id, q);
        p->precision = (int)o->precision;
    }
    if (capacity < (int)p->running.size())
        return fail(NMG_ERR_ARG, "result capacity below the requests in flight");
    // ---- one outer iteration for every member with work whose previous
    // iteration has finished (when none has, wait for the first that does);
    // members whose requests finished wait only for the copy-out of those
    // solutions.  Every early return below first reports the requests already
    // handed back in done[0..count), so a failing member never loses finished ones
    auto has_work = [](const nmg_pool_ctx::Member& m) { return !m.h->eng.queue.empty() || !m.h->eng.slot.empty(); };
    std::vector<char> ready(p->members.size(), 0);
    for (bool any_work = true, any_ready = false; any_work && !any_ready;) {
        any_work = false;
        for (size_t mi = 0; mi < p->members.size(); ++mi) {
            auto& m = p->members[mi];
            if (!has_work(m)) continue;
            any_work = true;
            hipError_t q = m.launched ? hipEventQuery(m.iter_done) : hipSuccess;
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return nmg::hip_fail(q, "hipEventQuery(iter_done)", __FILE__, __LINE__);
            ready[mi] = 1;
            any_ready = true;
        }
        if (any_work && !any_ready) std::this_thread::yield();
    }
    int count = 0;
    for (size_t mi = 0; mi < p->members.size(); ++mi) {
        auto& m = p->members[mi];
        if (!ready[mi]) continue;
        std::vector<nmg_request_result> out;
        const nmg_status st = nmg::engine_step(m.h, rtol, max_cycles, o, out, m.s, m.retired);
        if (st < 0) {
            *n_done = count;
            return st;
        }
        const hipError_t rec = hipEventRecord(m.iter_done, m.s);
        if (rec != hipSuccess) {
            *n_done = count;
            return nmg::hip_fail(rec, "hipEventRecord(iter_done)", __FILE__, __LINE__);
        }
        m.launched = true;
        if (out.empty()) continue;
        const hipError_t ev = hipEventSynchronize(m.retired);
        if (ev != hipSuccess) {
            *n_done = count;
            return nmg::hip_fail(ev, "hipEventSynchronize(retired)", __FILE__, __LINE__);
        }
        const double now = p->now_ms();
        for (auto& r : out) {
            if (count >= capacity) {
                *n_done = count;
                return fail(NMG_ERR_STATE, "more finished requests than the result capacity (a member handle "
                                           "received requests outside the pool)");
            }
            auto it = p->running.find(r.id);
            if (it != p->running.end()) {
                r.latency_ms = now - it->second.t_submit;
                p->in_flight -= it->second.bytes;
                p->running.erase(it);
            }
            done[count] = r;
            done_member[count] = (int)mi;
            ++count;
        }
    }
    if (p->running.empty()) p->precision = -1;
    *n_done = count;
    return NMG_OK;
}

nmg_status nmg_pool_pending(nmg_pool p, int* queued, int* active, size_t* bytes_in_flight) {
    if (!p) return fail(NMG_ERR_ARG, "null pool");
    if (queued) *queued = (int)p->queue.size();
    if (active) *active = (int)p->running.size();
    if (bytes_in_flight) *bytes_in_flight = p->in_flight;
    return NMG_OK;
}

nmg_status nmg_request_bytes(nmg_handle h, nmg_precision prec, size_t* bytes) {
    if (!h || !bytes) return fail(NMG_ERR_ARG, "null argument");
    if (prec != NMG_FP64 && prec != NMG_FP32 && prec != NMG_MIXED) return fail(NMG_ERR_ARG, "unknown precision");
    *bytes = nmg::request_bytes(h, prec);
    return NMG_OK;
}

}  // extern "C"
