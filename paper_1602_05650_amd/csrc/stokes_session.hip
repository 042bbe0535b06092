// Serving session: continuous batching of fiber mobility solves.
//
// A worker thread owns one HIP stream and a Batch (solver_batch.hpp).  Each
// loop it (1) retires cancelled requests, (2) admits queued requests in FIFO
// order while a slot is free and the request's device footprint fits the
// session's HBM arena, (3) runs one GMRES iteration for every request in
// flight with a single replay of the captured step graph, and (4) finalises
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

// First-fit allocator over one device allocation (offsets are 256-aligned).
class Arena {
public:
    int init(size_t bytes) {
        bytes = bytes & ~size_t(255);
        STOKES_HIP(hipMalloc(&base_, bytes));
        size_ = bytes;
        free_[0] = bytes;
        return STOKES_OK;
    }
    ~Arena() {
        if (base_) (void)hipFree(base_);
    }
    void* alloc(size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used_[off] = bytes;
                return static_cast<char*>(base_) + off;
            }
        }
        return nullptr;
    }
    void release(void* p) {
        const size_t off = static_cast<char*>(p) - static_cast<char*>(base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t len = u->second;
        used_.erase(u);
        auto nx = free_.lower_bound(off);   // first free block after the released one
        if (nx != free_.end() && nx->first == off + len) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += len;
                return;
            }
        }
        free_[off] = len;
    }
    size_t capacity() const { return size_; }

private:
    void* base_ = nullptr;
    size_t size_ = 0;
    std::map<size_t, size_t> free_, used_;
};

enum ReqState { QUEUED, RUNNING, DONE };

struct Request {
    uint64_t ticket = 0;
    int32_t n_fib = 0, npf = 0, k = 0;
    int64_t N = 0;
    double eps = 0, mu = 0, delta = 0;
    uint32_t opts = 0;            // STOKES_NONLOCAL | STOKES_PRECOND_BLOCK
    uint64_t tag = 0;
    size_t bytes = 0;
    double* host = nullptr;       // pinned: xyz | tan | rhs | flen | result
    ReqState state = QUEUED;
    bool cancel = false;
    bool claimed = false;         // a thread is inside stokes_session_wait for it
    int slot = -1;
    void* mem = nullptr;
    int j = 0;                    // iterations done
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
};

namespace stokes {

static void free_request(Request* r) {
    if (r->host) (void)hipHostFree(r->host);
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

static void worker_main(stokes_session* s) {
    (void)hipSetDevice(s->cfg.device);
    Batch& B = s->batch;
    std::vector<Request*>& slots = s->slot_req;
    for (;;) {
        std::vector<int> admitted;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                // retire cancelled requests (queued or in flight)
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
        // set-up of the newly admitted requests (device only; lock released)
        int rc = STOKES_OK;
        for (int q : admitted) {
            Request* r = slots[q];
            rc = B.attach(q, r->mem, r->n_fib, r->npf, r->k, r->eps, r->mu, 0.0, r->opts, r->delta,
                          r->xyz(), r->tan(),
                          r->flen(), r->rhs());
            if (rc) break;
        }
        if (!rc) rc = B.start(admitted);
        std::vector<int> iterating, finishing;
        std::vector<Batch::Part> parts;
        if (!rc) {
            for (int q = 0; q < (int)slots.size(); ++q) {
                Request* r = slots[q];
                if (!r) continue;
                const bool fresh = std::find(admitted.begin(), admitted.end(), q) != admitted.end();
                if (fresh) {
                    r->j = 0;
                    r->sl_done = 0;
                    r->sl_quota = step_quota(B.desc(q), s->cfg.step_pairs);
                    r->st.residual = B.status(q)[2];
                    if (B.status(q)[3] != 0.0) {   // zero right-hand side
                        finishing.push_back(q);
                        continue;
                    }
                }
                B.desc(q).j = r->j;
                iterating.push_back(q);
            }
            if (s->inject_fault.exchange(false) && !iterating.empty()) {
                // forced failure of this step: fail the requests in flight, keep serving
                std::lock_guard<std::mutex> lk(s->mu);
                set_error("injected step failure");
                for (int q : iterating) finish(s, slots[q], STOKES_E_DEVICE);
                iterating.clear();
                s->cv_done.notify_all();
            }
            for (int q : iterating) {
                Request* r = slots[q];
                const int32_t n = B.desc(q).n_items_sl;
                parts.push_back({q, r->sl_done, std::min(r->sl_quota, n - r->sl_done)});
            }
            rc = B.step_parts(parts);
        }
        if (!rc) {
            for (const Batch::Part& p : parts) {
                Request* r = slots[p.slot];
                r->sl_done += p.sl_count;
                if (r->sl_done < B.desc(p.slot).n_items_sl) continue;   // matvec not complete
                r->sl_done = 0;
                r->j += 1;
                r->st.residual = B.status(p.slot)[2];
                if (r->j >= r->k || B.status(p.slot)[3] != 0.0) finishing.push_back(p.slot);
            }
            for (int q : finishing) B.desc(q).j = slots[q]->j;
            rc = B.finalize(finishing);
        }
        if (!rc) {
            for (int q : finishing) {
                Request* r = slots[q];
                hipError_t e = hipMemcpyAsync(r->result(), B.desc(q).x, 3 * r->N * sizeof(double),
                                              hipMemcpyDeviceToHost, s->st);
                if (e != hipSuccess) { rc = hip_fail(e, "hipMemcpyAsync(result)"); break; }
            }
            if (!rc && !finishing.empty()) {
                hipError_t e = hipStreamSynchronize(s->st);
                if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
            }
        }
        std::lock_guard<std::mutex> lk(s->mu);
        if (rc) {
            // a device error fails every request in flight; the session stops admitting
            s->worker_rc = rc;
            for (Request*& r : slots)
                if (r) finish(s, r, rc);
            for (Request* r : s->queue) finish(s, r, rc);
            s->queue.clear();
            s->stop = true;
            s->cv_done.notify_all();
            return;
        }
        for (int q : finishing) finish(s, slots[q], STOKES_OK);
        if (!finishing.empty()) s->cv_done.notify_all();
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
    if (!rc) {
        rc = s->arena.init((size_t)cfg->hbm_budget_bytes);
        if (rc) rc = fail(STOKES_E_NOMEM, std::string("stokes_session_create: HBM arena: ") + stokes_last_error());
    }
    (void)hipSetDevice(cur);
    if (rc) {
        if (s->st) (void)hipStreamDestroy(s->st);
        delete s;
        return rc;
    }
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
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(s->cfg.device);
    (void)hipStreamSynchronize(s->st);
    const int rc = s->worker_rc;
    hipStream_t st = s->st;
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
