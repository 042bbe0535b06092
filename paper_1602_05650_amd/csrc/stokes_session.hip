// Serving session: continuous batching of fiber mobility solves.
//
// A worker thread owns one HIP stream and a Batch (solver_batch.hpp).  Each
// loop it (1) retires cancelled requests, (2) admits queued requests in FIFO
// order while a slot is free and the request's device footprint fits the
// session's HBM arena, (3) runs one GMRES iteration for every request in
// flight with a single replay of the captured step graph (requests whose u_bar
// goes through a treecode plan run their iteration with launches of their own right
// after it), and (4) finalises
// the requests that used their iteration budget (or broke down), copies their
// solutions to host memory and frees their slots.  Requests therefore join
// and leave the batch between steps while the others keep iterating.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <string>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "solver_batch.hpp"

namespace stokes {

static int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

// One device allocation, placed by the first-fit RangeAllocator (host_logic.hpp).
class Arena {
public:
    int init(size_t bytes) {
        bytes = bytes & ~size_t(255);
        STOKES_HIP(hipMalloc(&base_, bytes));
        ranges_.reset(bytes);
        return STOKES_OK;
    }
    ~Arena() {
        if (base_) (void)hipFree(base_);
    }
    void* alloc(size_t bytes) {
        const size_t off = ranges_.alloc(bytes);
        return off == SIZE_MAX ? nullptr : static_cast<char*>(base_) + off;
    }
    void release(void* p) { ranges_.release(static_cast<char*>(p) - static_cast<char*>(base_)); }
    bool fits(size_t bytes) const { return ranges_.fits(bytes); }
    size_t capacity() const { return ranges_.capacity(); }

private:
    void* base_ = nullptr;
    RangeAllocator ranges_;
};

enum ReqState { QUEUED, RUNNING, DONE };

struct Request {
    uint64_t ticket = 0;
    int32_t n_fib = 0, npf = 0, k = 0;
    int64_t N = 0;
    double eps = 0, mu = 0, delta = 0;
    uint32_t opts = 0;            // STOKES_NONLOCAL | STOKES_PRECOND_BLOCK
    bool far = false;             // u_bar through a treecode plan (farp), built at admission
    stokes_far farp{};
    FarPlan* fplan = nullptr;
    uint64_t tag = 0;
    size_t bytes = 0;
    double* host = nullptr;       // pinned: xyz | tan | rhs | flen | result
    ReqState state = QUEUED;
    bool cancel = false;
    bool claimed = false;         // a thread is inside stokes_session_wait for it
    int slot = -1;
    void* mem = nullptr;
    int j = 0;                    // iterations enqueued (complete once their step is)
    bool final_queued = false;    // the solution and its copy to the host are enqueued
    int32_t sl_done = 0;          // single-layer items of iteration j already summed
    int32_t sl_quota = 0;         // single-layer items per step
    stokes_solve_stats st{};
    double* xyz() { return host; }
    double* tan() { return host + 3 * N; }
    double* rhs() { return host + 6 * N; }
    double* flen() { return host + 9 * N; }
    double* result() { return host + 9 * N + n_fib; }
};

}  // namespace stokes

struct stokes_session {
    stokes_session_cfg cfg{};
    hipStream_t st = nullptr;
    stokes::Batch batch;
    stokes::Arena arena;
    // Status rows of the last two enqueued steps (pinned) and the event after each
    // step's work: the worker enqueues step t before it reads step t-1's status.
    double* stat_buf[2] = {nullptr, nullptr};
    hipEvent_t stat_ev[2] = {nullptr, nullptr};
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::atomic<bool> inject_fault{false};
    int waiters = 0;
    int worker_rc = STOKES_OK;
    uint64_t next_ticket = 1;
    std::deque<stokes::Request*> queue;
    std::map<uint64_t, stokes::Request*> reqs;
    std::vector<stokes::Request*> slot_req;
    // tree plans of finished requests, freed by the worker outside the lock (freeing
    // device memory waits for the device)
    std::vector<stokes::FarPlan*> dead_plans;
};

namespace stokes {

static void free_request(Request* r) {
    if (r->host) (void)hipHostFree(r->host);
    delete r->fplan;
    delete r;
}

// Mark a request finished (called with the lock held).
static void finish(stokes_session* s, Request* r, int status) {
    r->state = DONE;
    r->st.status = status;
    r->st.t_finish_ns = now_ns();
    r->st.iters = r->j;
    if (r->slot >= 0) {
        s->slot_req[r->slot] = nullptr;
        r->slot = -1;
    }
    if (r->mem) {
        s->arena.release(r->mem);
        r->mem = nullptr;
    }
    if (r->fplan) s->dead_plans.push_back(r->fplan);   // no step still reads it: see the callers
    r->fplan = nullptr;
}

// Free the tree plans of finished requests (lock not held).
static void free_dead_plans(stokes_session* s) {
    std::vector<FarPlan*> dead;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        dead.swap(s->dead_plans);
    }
    for (FarPlan* p : dead) delete p;
}

// Single-layer items a request takes per step: its pair budget over the pairs
// of one item (target block x source chunk), at least one item.
static int32_t step_quota(const SlotDesc& d, int64_t step_pairs) {
    if (step_pairs == 0) step_pairs = STOKES_STEP_PAIRS_DEFAULT;
    if (step_pairs < 0 || d.n_items_sl <= 0) return std::max<int32_t>(1, d.n_items_sl);
    const double pairs_per_item = (double)d.N * (double)d.N / d.n_items_sl;
    const double q = std::floor((double)step_pairs / std::max(1.0, pairs_per_item));
    return (int32_t)std::max(1.0, std::min<double>(q, d.n_items_sl));
}

// A step on the stream whose status the worker has not read yet.
struct Pending {
    bool valid = false;
    int buf = 0;                                // stat_buf / stat_ev index
    std::vector<std::pair<int, int>> done;      // (slot, iteration the step completed)
    std::vector<int> final_slots;               // slots whose solution copy the event covers
};

// Would the FIFO head be admitted now (a free slot and room in the arena)?  Lock held.
static bool admissible(stokes_session* s) {
    if (s->queue.empty()) return false;
    bool slot = false;
    for (Request* r : s->slot_req) slot |= (r == nullptr);
    return slot && s->arena.fits(s->queue.front()->bytes);
}

// Wait for a pending step and take in its status: residuals, exact breakdowns (the
// request's solution is formed from the iterations before the breakdown; the extra
// iteration a lagging host enqueued for it touches only entries beyond them), and the
// requests whose solution copy the step's event covers.  `next` is the step enqueued
// after it (a broken-down request is taken out of its finishing list).
static int complete_pending(stokes_session* s, Pending& P, Pending* next) {
    if (!P.valid) return STOKES_OK;
    P.valid = false;
    STOKES_HIP(hipEventSynchronize(s->stat_ev[P.buf]));
    const double* st = s->stat_buf[P.buf];
    Batch& B = s->batch;
    std::vector<int> broken;
    for (const auto& dq : P.done) {
        const int q = dq.first;
        Request* r = s->slot_req[q];
        if (!r) continue;
        r->st.residual = st[NSTAT * q + 2];
        if (st[NSTAT * q + 3] != 0.0 && std::find(P.final_slots.begin(), P.final_slots.end(), q) ==
                                            P.final_slots.end()) {
            r->j = dq.second + 1;
            broken.push_back(q);
        }
    }
    if (!broken.empty()) {   // rare: finish them now, synchronously
        for (int q : broken) B.desc(q).j = s->slot_req[q]->j;
        if (int rc = B.finalize(broken)) return rc;
        for (int q : broken) {
            Request* r = s->slot_req[q];
            STOKES_HIP(hipMemcpyAsync(r->result(), B.desc(q).x, 3 * r->N * sizeof(double), hipMemcpyDeviceToHost,
                                      s->st));
            if (next) next->final_slots.erase(std::remove(next->final_slots.begin(), next->final_slots.end(), q),
                                              next->final_slots.end());
        }
        STOKES_HIP(hipStreamSynchronize(s->st));
    }
    std::lock_guard<std::mutex> lk(s->mu);
    for (int q : P.final_slots)
        if (s->slot_req[q]) finish(s, s->slot_req[q], STOKES_OK);
    for (int q : broken)
        if (s->slot_req[q]) finish(s, s->slot_req[q], STOKES_OK);
    if (!P.final_slots.empty() || !broken.empty()) s->cv_done.notify_all();
    return STOKES_OK;
}

// Fail every request (device error): the session stops admitting.  Lock held.
static void fail_all(stokes_session* s, int rc) {
    s->worker_rc = rc;
    for (Request*& r : s->slot_req)
        if (r) finish(s, r, rc);
    for (Request* r : s->queue) finish(s, r, rc);
    s->queue.clear();
    s->stop = true;
    s->cv_done.notify_all();
}

static void worker_main(stokes_session* s) {
    (void)hipSetDevice(s->cfg.device);
    Batch& B = s->batch;
    std::vector<Request*>& slots = s->slot_req;
    Pending pend;
    int next_buf = 0;
    for (;;) {
        free_dead_plans(s);
        // Admissions, cancellations of running requests, fault injection and stopping
        // need an empty pipeline (memory of a finished request is reused only after its
        // last step): drain the pending step first when one of them is due.
        bool drain = false;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            bool retired = false;
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                if ((*it)->cancel) {
                    finish(s, *it, STOKES_E_CANCELED);
                    it = s->queue.erase(it);
                    retired = true;
                } else {
                    ++it;
                }
            }
            if (retired) s->cv_done.notify_all();
            bool running_cancel = false;
            for (Request* r : slots) running_cancel |= (r && r->cancel);
            drain = pend.valid && (s->stop || running_cancel || s->inject_fault.load() || admissible(s));
        }
        if (drain) {
            if (int rc = complete_pending(s, pend, nullptr)) {
                std::lock_guard<std::mutex> lk(s->mu);
                fail_all(s, rc);
                return;
            }
        }
        std::vector<int> admitted;
        if (!pend.valid) {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                for (auto it = s->queue.begin(); it != s->queue.end();) {
                    if ((*it)->cancel) {
                        finish(s, *it, STOKES_E_CANCELED);
                        it = s->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
                for (Request*& r : slots)
                    if (r && r->cancel) finish(s, r, STOKES_E_CANCELED);
                if (s->stop) break;
                if (s->inject_fault.exchange(false)) {
                    // forced failure of this step: fail the requests in flight, keep serving
                    bool any = false;
                    for (Request* r : slots) any |= (r != nullptr);
                    if (any) {
                        set_error("injected step failure");
                        for (Request*& r : slots)
                            if (r) finish(s, r, STOKES_E_DEVICE);
                        s->cv_done.notify_all();
                    }
                }
                // FIFO admission by slot and device-memory footprint
                while (!s->queue.empty()) {
                    Request* r = s->queue.front();
                    int free_slot = -1;
                    for (int q = 0; q < (int)slots.size(); ++q)
                        if (!slots[q]) { free_slot = q; break; }
                    if (free_slot < 0) break;
                    void* mem = s->arena.alloc(r->bytes);
                    if (!mem) break;
                    s->queue.pop_front();
                    r->mem = mem;
                    r->slot = free_slot;
                    r->state = RUNNING;
                    r->st.t_admit_ns = now_ns();
                    slots[free_slot] = r;
                    admitted.push_back(free_slot);
                }
                bool any = !admitted.empty();
                for (Request* r : slots) any |= (r != nullptr);
                if (any) break;
                s->cv_done.notify_all();
                s->cv_work.wait(lk);
            }
            if (s->stop) {
                for (Request*& r : slots)
                    if (r) finish(s, r, STOKES_E_CANCELED);
                for (Request* r : s->queue) finish(s, r, STOKES_E_CANCELED);
                s->queue.clear();
                s->cv_done.notify_all();
                return;
            }
            s->cv_done.notify_all();
        }
        // set-up of the newly admitted requests (the pipeline is empty; lock released)
        Range range("stokes_session step");
        int rc = STOKES_OK;
        for (int q : admitted) {
            Request* r = slots[q];
            rc = B.attach(q, r->mem, r->n_fib, r->npf, r->k, r->eps, r->mu, 0.0, r->far ? r->opts | OPT_FAR : r->opts,
                          r->delta, r->xyz(), r->tan(), r->flen(), r->rhs());
            if (!rc && r->far) {   // the tree plan of the request's nodes (synchronous)
                r->fplan = new FarPlan();
                rc = r->fplan->make(r->N, B.desc(q).xyz, r->farp, s->st);
            }
            if (rc) break;
        }
        if (!rc) rc = B.start(admitted);   // synchronous: reads beta and the breakdown flag
        Pending cur;
        cur.buf = next_buf;
        std::vector<Batch::Part> parts;
        std::vector<int> far_slots;   // treecode requests: a whole iteration each step
        std::vector<int> zero_rhs;
        if (!rc) {
            for (int q = 0; q < (int)slots.size(); ++q) {
                Request* r = slots[q];
                if (!r || r->final_queued) continue;
                if (std::find(admitted.begin(), admitted.end(), q) != admitted.end()) {
                    r->j = 0;
                    r->sl_done = 0;
                    r->sl_quota = step_quota(B.desc(q), s->cfg.step_pairs);
                    r->st.residual = B.status(q)[2];
                    if (B.status(q)[3] != 0.0) {   // zero right-hand side: x = 0
                        zero_rhs.push_back(q);
                        continue;
                    }
                }
                B.desc(q).j = r->j;
                if (r->far) {
                    far_slots.push_back(q);
                    continue;
                }
                const int32_t n = B.desc(q).n_items_sl;
                parts.push_back({q, r->sl_done, std::min(r->sl_quota, n - r->sl_done)});
            }
            if (parts.empty() && far_slots.empty() && zero_rhs.empty()) {
                // nothing left to step (every request in a slot has its solution queued):
                // take in the pending step and go back to waiting for work
                rc = complete_pending(s, pend, nullptr);
                if (rc) {
                    (void)hipStreamSynchronize(s->st);
                    std::lock_guard<std::mutex> lk(s->mu);
                    fail_all(s, rc);
                    return;
                }
                continue;
            }
            rc = B.step_parts_nowait(parts);
            // the treecode requests' iteration after the step's graph, on the same stream:
            // z = M^{-1} v_j, u_bar through the tree into partial row 0, reduction,
            // Gram-Schmidt and Givens (the own fiber excluded, as in the direct sum)
            const uint32_t tflags = (s->cfg.flags & (STOKES_PREC_MIXED | STOKES_NO_DOUBLET)) | STOKES_EXCL_SAME_FIBER;
            auto far_sum = [&](int q) {
                const SlotDesc& d = B.desc(q);
                const Request* r = slots[q];
                return stokes_tree_sl_eval(r->fplan->t, d.z, d.wq, d.fib, d.n_fib, d.flen, r->mu, r->eps, 0.0,
                                           tflags, d.partial, s->st);
            };
            if (!rc) rc = B.step_external_nowait(far_slots, far_sum);
        }
        if (!rc && (!parts.empty() || !far_slots.empty())) rc = B.copy_status_async(s->stat_buf[cur.buf]);
        if (!rc) {
            std::vector<int> finishing = zero_rhs;
            for (int q : far_slots) {
                Request* r = slots[q];
                cur.done.push_back({q, r->j});
                r->j += 1;
                if (r->j >= r->k) finishing.push_back(q);
            }
            for (const Batch::Part& p : parts) {
                Request* r = slots[p.slot];
                r->sl_done += p.sl_count;
                if (r->sl_done < B.desc(p.slot).n_items_sl) continue;   // matvec not complete
                r->sl_done = 0;
                cur.done.push_back({p.slot, r->j});
                r->j += 1;
                if (r->j >= r->k) finishing.push_back(p.slot);
            }
            for (int q : finishing) {
                B.desc(q).j = slots[q]->j;
                slots[q]->final_queued = true;
            }
            rc = B.finalize(finishing);
            for (int q : finishing) {
                if (rc) break;
                Request* r = slots[q];
                hipError_t e = hipMemcpyAsync(r->result(), B.desc(q).x, 3 * r->N * sizeof(double),
                                              hipMemcpyDeviceToHost, s->st);
                if (e != hipSuccess) rc = hip_fail(e, "hipMemcpyAsync(result)");
            }
            cur.final_slots = finishing;
        }
        if (!rc) {
            hipError_t e = hipEventRecord(s->stat_ev[cur.buf], s->st);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventRecord");
        }
        cur.valid = true;
        // the previous step's status, read while this one runs
        if (!rc) rc = complete_pending(s, pend, &cur);
        if (rc) {
            (void)hipStreamSynchronize(s->st);
            std::lock_guard<std::mutex> lk(s->mu);
            fail_all(s, rc);
            return;
        }
        pend = cur;
        next_buf ^= 1;
    }
}

}  // namespace stokes

using namespace stokes;

extern "C" int stokes_session_create(const stokes_session_cfg* cfg, stokes_session** out) {
    if (!cfg || !out) return fail(STOKES_E_INVAL, "stokes_session_create: null argument");
    if (cfg->hbm_budget_bytes <= 0) return fail(STOKES_E_INVAL, "stokes_session_create: hbm_budget_bytes <= 0");
    if (cfg->max_slots < 1 || cfg->max_slots > MAX_SLOTS)
        return fail(STOKES_E_INVAL, "stokes_session_create: max_slots out of range");
    if (cfg->max_queue < 1) return fail(STOKES_E_INVAL, "stokes_session_create: max_queue < 1");
    if (cfg->flags & ~(STOKES_PREC_MIXED | STOKES_NO_DOUBLET))
        return fail(STOKES_E_INVAL, "stokes_session_create: unknown flag bits");
    int ndev = 0;
    STOKES_HIP(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev)
        return fail(STOKES_E_INVAL, "stokes_session_create: no such device");
    int cur = 0;
    STOKES_HIP(hipGetDevice(&cur));
    STOKES_HIP(hipSetDevice(cfg->device));
    stokes_session* s = new stokes_session();
    s->cfg = *cfg;
    s->slot_req.assign(cfg->max_slots, nullptr);
    int rc = STOKES_OK;
    hipError_t e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
    if (e != hipSuccess) rc = hip_fail(e, "hipStreamCreateWithFlags");
    if (!rc) rc = s->batch.init(s->st, cfg->flags & STOKES_PREC_MIXED,
                                !(cfg->flags & STOKES_NO_DOUBLET), true);
    for (int b = 0; b < 2 && !rc; ++b) {
        e = hipHostMalloc((void**)&s->stat_buf[b], sizeof(double) * NSTAT * MAX_SLOTS, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->stat_ev[b], hipEventDisableTiming);
        if (e != hipSuccess) rc = hip_fail(e, "stokes_session_create: status buffers");
    }
    if (!rc) {
        rc = s->arena.init((size_t)cfg->hbm_budget_bytes);
        if (rc) rc = fail(STOKES_E_NOMEM, std::string("stokes_session_create: HBM arena: ") + stokes_last_error());
    }
    if (rc) {
        for (int b = 0; b < 2; ++b) {
            if (s->stat_ev[b]) (void)hipEventDestroy(s->stat_ev[b]);
            if (s->stat_buf[b]) (void)hipHostFree(s->stat_buf[b]);
        }
        hipStream_t st = s->st;
        delete s;   // the batch waits for its stream before it releases its tables
        if (st) (void)hipStreamDestroy(st);
        (void)hipSetDevice(cur);
        return rc;
    }
    (void)hipSetDevice(cur);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return STOKES_OK;
}

extern "C" int stokes_session_submit(stokes_session* s, const stokes_solve_req* req,
                                     uint64_t* ticket) {
    if (!s || !req || !ticket) return fail(STOKES_E_INVAL, "stokes_session_submit: null argument");
    if (req->n_fib < 1 || req->nodes_per_fib < 2 || req->nodes_per_fib > 64)
        return fail(STOKES_E_INVAL, "stokes_session_submit: need n_fib >= 1 and 2 <= nodes_per_fib <= 64");
    if (req->iters < 1 || req->iters > STOKES_MAX_ITERS)
        return fail(STOKES_E_INVAL, "stokes_session_submit: iters out of range");
    if (!(req->mu > 0.0) || !(req->eps > 0.0 && req->eps < 0.5))
        return fail(STOKES_E_INVAL, "stokes_session_submit: bad mu or eps");
    if (!req->xyz || !req->tangent || !req->fiber_len || !req->rhs)
        return fail(STOKES_E_INVAL, "stokes_session_submit: null array");
    const int64_t N = (int64_t)req->n_fib * req->nodes_per_fib;
    if (N >= (int64_t)1 << 30) return fail(STOKES_E_INVAL, "stokes_session_submit: too many nodes");
    for (int64_t i = 0; i < 3 * N; ++i)
        if (!std::isfinite(req->xyz[i]) || !std::isfinite(req->tangent[i]) || !std::isfinite(req->rhs[i]))
            return fail(STOKES_E_NONFINITE, "stokes_session_submit: non-finite input");
    for (int32_t f = 0; f < req->n_fib; ++f)
        if (!std::isfinite(req->fiber_len[f]) || !(req->fiber_len[f] > 0.0))
            return fail(STOKES_E_INVAL, "stokes_session_submit: fiber lengths must be finite and > 0");
    const bool mixed = s->cfg.flags & STOKES_PREC_MIXED;
    if (req->flags & ~(STOKES_NONLOCAL | STOKES_PRECOND_BLOCK))
        return fail(STOKES_E_INVAL, "stokes_session_submit: unknown request flag bits");
    if ((req->flags & STOKES_NONLOCAL) && (!(req->delta > 0.0) || !std::isfinite(req->delta)))
        return fail(STOKES_E_INVAL, "stokes_session_submit: delta must be finite and > 0 with STOKES_NONLOCAL");
    if (int rc = check_far(req->far, "stokes_session_submit")) return rc;
    const size_t bytes =
        slot_plan(req->n_fib, req->nodes_per_fib, req->iters, mixed, req->flags).bytes;
    if (bytes > s->arena.capacity())
        return fail(STOKES_E_NOMEM, "stokes_session_submit: request needs " + std::to_string(bytes) +
                                        " bytes, more than the session budget");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(s->worker_rc ? s->worker_rc : STOKES_E_CANCELED,
                                 "stokes_session_submit: session stopped");
        if ((int)s->queue.size() >= s->cfg.max_queue)
            return fail(STOKES_E_BUSY, "stokes_session_submit: queue full");
    }
    Request* r = new Request();
    r->n_fib = req->n_fib;
    r->npf = req->nodes_per_fib;
    r->k = req->iters;
    r->N = N;
    r->eps = req->eps;
    r->mu = req->mu;
    r->opts = req->flags;
    r->delta = req->delta;
    if (req->far) {
        r->far = true;
        r->farp = *req->far;
    }
    r->tag = req->tag;
    r->bytes = bytes;
    const size_t hb = sizeof(double) * (12 * N + r->n_fib);
    hipError_t e = hipHostMalloc((void**)&r->host, hb, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete r;
        return fail(STOKES_E_NOMEM, "stokes_session_submit: pinned host buffer");
    }
    memcpy(r->xyz(), req->xyz, 3 * N * sizeof(double));
    memcpy(r->tan(), req->tangent, 3 * N * sizeof(double));
    memcpy(r->rhs(), req->rhs, 3 * N * sizeof(double));
    memcpy(r->flen(), req->fiber_len, r->n_fib * sizeof(double));
    r->st.tag = req->tag;
    r->st.t_submit_ns = now_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            free_request(r);
            return fail(STOKES_E_CANCELED, "stokes_session_submit: session stopped");
        }
        r->ticket = s->next_ticket++;
        s->reqs[r->ticket] = r;
        s->queue.push_back(r);
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return STOKES_OK;
}

extern "C" int stokes_session_wait(stokes_session* s, uint64_t ticket, double* f_out,
                                   stokes_solve_stats* st, int32_t timeout_ms) {
    if (!s) return fail(STOKES_E_INVAL, "stokes_session_wait: null session");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(STOKES_E_NOTFOUND, "stokes_session_wait: unknown ticket");
    Request* r = it->second;
    if (r->claimed) return fail(STOKES_E_BUSY, "stokes_session_wait: another thread waits for this ticket");
    r->claimed = true;
    s->waiters++;
    auto ready = [&] { return r->state == DONE; };
    bool ok = true;
    if (timeout_ms < 0)
        s->cv_done.wait(lk, ready);
    else
        ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    s->waiters--;
    if (!ok) {
        r->claimed = false;
        s->cv_done.notify_all();
        return fail(STOKES_E_TIMEOUT, "stokes_session_wait: timeout");
    }
    const int status = r->st.status;
    if (st) *st = r->st;
    if (f_out && status == STOKES_OK) memcpy(f_out, r->result(), 3 * r->N * sizeof(double));
    s->reqs.erase(ticket);
    free_request(r);
    s->cv_done.notify_all();
    if (status != STOKES_OK) return fail(status, "stokes_session_wait: request failed or was cancelled");
    return STOKES_OK;
}

extern "C" int stokes_session_cancel(stokes_session* s, uint64_t ticket) {
    if (!s) return fail(STOKES_E_INVAL, "stokes_session_cancel: null session");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return fail(STOKES_E_NOTFOUND, "stokes_session_cancel: unknown ticket");
        if (it->second->state != DONE) it->second->cancel = true;
    }
    s->cv_work.notify_one();
    return STOKES_OK;
}

extern "C" int stokes_session_destroy(stokes_session* s) {
    if (!s) return fail(STOKES_E_INVAL, "stokes_session_destroy: null session");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    {
        // wake waiters (their requests are now finished) and let them leave
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.notify_all();
        s->cv_done.wait(lk, [&] { return s->waiters == 0; });
        for (auto& kv : s->reqs) free_request(kv.second);
        s->reqs.clear();
    }
    free_dead_plans(s);
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->cfg.device);
    (void)hipStreamSynchronize(s->st);
    const int rc = s->worker_rc;
    hipStream_t st = s->st;
    for (int b = 0; b < 2; ++b) {
        if (s->stat_ev[b]) (void)hipEventDestroy(s->stat_ev[b]);
        if (s->stat_buf[b]) (void)hipHostFree(s->stat_buf[b]);
    }
    delete s;   // batch and arena free their device memory
    (void)hipStreamDestroy(st);
    (void)hipSetDevice(cur);
    return rc ? rc : STOKES_OK;
}

extern "C" int64_t stokes_solve_footprint(int32_t n_fib, int32_t nodes_per_fib, int32_t iters,
                                          uint32_t flags) {
    if (n_fib < 1 || nodes_per_fib < 2 || nodes_per_fib > 64 || iters < 1 || iters > STOKES_MAX_ITERS)
        return 0;
    if ((int64_t)n_fib * nodes_per_fib >= (int64_t)1 << 30) return 0;
    return (int64_t)slot_plan(n_fib, nodes_per_fib, iters, flags & STOKES_PREC_MIXED,
                              flags & STOKES_PRECOND_BLOCK).bytes;
}

extern "C" int stokes_session_inject_fault(stokes_session* s) {
    if (!s) return fail(STOKES_E_INVAL, "stokes_session_inject_fault: null session");
    s->inject_fault.store(true);
    s->cv_work.notify_one();
    return STOKES_OK;
}
