// Batched FP64 GMRES for the fiber mobility problem (shared by the one-shot
// solve and the serving session).
//
// Every request lives in a "slot": its geometry, Krylov basis and small
// Hessenberg state in device memory, described by a SlotDesc in a device
// table.  Each GMRES step is a fixed sequence of kernels; every kernel walks a
// work list of (slot, item) pairs with a grid-stride loop, so one launch
// serves all requests in flight and the sequence can be captured once in a
// HIP graph (the tables live at fixed addresses; only their contents change).
// A slot's arithmetic depends only on its own data and on a partition fixed
// by its own sizes, never on the other slots: results are the same alone and
// in any batch, bit for bit.
#pragma once

#include <vector>

#include "stokes_internal.hpp"
#include "sum_device.hpp"

namespace stokes {

constexpr int MAX_SLOTS = 256;
constexpr int KMAX = STOKES_MAX_ITERS;

struct SlotDesc {
    int32_t N;            // nodes
    int32_t n_fib, npf;   // fibers, nodes per fiber
    int32_t k;            // iteration budget
    int32_t j;            // iteration computed this step (finalize: iterations done)
    int32_t B;            // dot-product blocks (fixed by N)
    int32_t n_items_vec;  // ceil(3N / 256)
    int32_t n_items_node; // ceil(N / 256)
    int32_t n_items_sl;   // SL work items (target blocks x chunks)
    int32_t sid;          // slot index (row of the status table)
    uint32_t opts;        // STOKES_NONLOCAL | STOKES_PRECOND_BLOCK
    int32_t pad0;
    double eps, mu, kappa, pref, near_r;
    double delta;         // K_delta regularisation
    SumArgs sl;           // single-layer sum over the slot's own nodes
    const double* xyz;    // [3][N]
    const double* tan;    // [3][N]
    const double* flen;   // [n_fib]
    const double* rhs;    // [3][N]
    int32_t* fib;         // [N]
    double* wq;           // [N] Clenshaw-Curtis weight x L/2
    double* sarc;         // [N] arc length s = (L/2)(1 + alpha_k)
    double* binv;         // [n_fib][3 npf][3 npf] inverse self blocks, column-major
                          // (row and column index c npf + k), or null
    double* V;            // [(k+1)][3N]
    double* z;            // [3][N]  M^{-1} v_j
    double* w;            // [3][N]
    double* x;            // [3][N]  solution
    double* dotp;         // [(k+1)][B] dot partials
    double* normp;        // [B]
    double* hA;           // [k+1]
    double* hB;           // [k+1]
    double* H;            // [(k+1) x k], column-major, ld = k+1
    double* cs;           // [k]
    double* sn;           // [k]
    double* g;            // [k+1]
    double* y;            // [k]
    SrcSL64* s64;
    SrcSL32* s32;
    float* near_t;
    Tile* tiles;
    int2* excl;
    double* partial;
};

// Work list of one kernel: slots taking part, the prefix sum of their items and,
// per slot, the index of its first item (nonzero only when a slot's single-layer
// sum is split over several steps).
struct WorkList {
    int32_t n;
    int32_t pad;
    int32_t slot[MAX_SLOTS];
    int64_t prefix[MAX_SLOTS + 1];
    int64_t base[MAX_SLOTS];
};

enum WL {
    WL_PRE = 0,  // z = M^{-1} v_j, pack sources          items: ceil(N/256)
    WL_SL,       // single-layer sum                       items: target blocks x chunks
    WL_RED,      // w = M z + sum of chunk partials        items: ceil(N/256)
    WL_DOT,      // partial dots of V[0..j] with w         items: B
    WL_ONE,      // one block per slot (reductions, Givens) items: 1
    WL_VEC,      // elementwise over 3N                    items: ceil(3N/256)
    WL_FIB,      // one block per fiber (block-Jacobi set-up) items: n_fib or 0
    WL_COUNT
};

struct StepTables {
    WorkList wl[WL_COUNT];
};

// Status row per slot, read back after every step: hn, beta, residual, breakdown.
constexpr int NSTAT = 4;

struct SlotPlan {
    Partition P;
    int32_t B;
    size_t bytes;
};
SlotPlan slot_plan(int32_t n_fib, int32_t npf, int32_t k, bool mixed, uint32_t opts);
// Bytes of a generic-vector slot (attach_vector).
size_t vector_plan_bytes(int64_t n_vec, int32_t k);

// The fixed-size resources of a Batch: pinned host tables, the upload ring, two lagged
// status rows, events and the device tables.  Made once and kept per device in a free
// list (batch_res_acquire / batch_res_release): a later Batch takes them back instead
// of making some twenty pinned allocations again.
struct BatchRes;
constexpr int UPLOAD_RING = 8;   // pinned table snapshots of a Batch's upload ring

class Batch {
public:
    Batch() = default;
    ~Batch();
    Batch(const Batch&) = delete;
    Batch& operator=(const Batch&) = delete;
    int init(hipStream_t st, bool mixed, bool doublet, bool use_graph);
    // Lay a request out in `mem` (slot_plan bytes) and copy its inputs there
    // (hipMemcpyDefault: host inputs must be pinned for the copy to be async).
    int attach(int s, void* mem, int32_t n_fib, int32_t npf, int32_t k, double eps, double mu,
               double near_r, uint32_t opts, double delta, const double* xyz,
               const double* tan, const double* flen, const double* rhs);
    // Geometry set-up (and the inverted fiber blocks), beta = |rhs| and v_0 for
    // newly attached slots.
    int start(const std::vector<int>& slots);
    // One GMRES iteration for every listed slot, then read the status rows back.
    int step(const std::vector<int>& slots);
    // Part of one GMRES iteration per listed slot: single-layer items
    // [sl_begin, sl_begin + sl_count) of the slot's current iteration.  The part
    // with sl_begin == 0 also forms z = M^{-1} v_j and the source pack; the part
    // that reaches the last item also finishes the iteration (reduction,
    // Gram-Schmidt, Givens) and only for those slots is the status row fresh.
    // The items write disjoint partials, so the split does not change a bit.
    struct Part {
        int slot;
        int32_t sl_begin, sl_count;
    };
    int step_parts(const std::vector<Part>& parts);
    // One GMRES iteration of slots attached with OPT_FAR: z = M^{-1} v_j, then `sl(slot)`
    // writes each slot's single-layer sum (3 x N, the own fiber excluded) into its
    // partial row 0, then the reduction, Gram-Schmidt and Givens; status read back.
    template <class F>
    int step_external(const std::vector<int>& slots, F&& sl) {
        if (slots.empty()) return STOKES_OK;
        if (int rc = launch_pre(slots)) return rc;
        for (int q : slots)
            if (int rc = sl(q)) return rc;
        if (int rc = launch_red_ortho(slots)) return rc;
        return read_status();
    }
    // step_external without reading the status rows back: only enqueued (after whatever
    // the stream holds, e.g. the graph of the other slots' step).
    template <class F>
    int step_external_nowait(const std::vector<int>& slots, F&& sl) {
        if (slots.empty()) return STOKES_OK;
        if (int rc = launch_pre(slots)) return rc;
        for (int q : slots)
            if (int rc = sl(q)) return rc;
        return launch_red_ortho(slots);
    }
    // step_parts without reading the status rows back: the step is only enqueued.
    // copy_status_async then enqueues the copy of the status rows into `dst` (pinned
    // host memory of MAX_SLOTS * NSTAT doubles), valid once the stream reaches it; on
    // stream s (a capturing stream), or on the Batch's stream when s is null.
    int step_parts_nowait(const std::vector<Part>& parts);
    int copy_status_async(double* dst, hipStream_t s = nullptr);
    // Solutions of the listed slots into their x buffers (iterations done in desc.j).
    int finalize(const std::vector<int>& slots);

    // ---- GMRES for an operator applied by the caller (generic vectors) -------
    // A slot holding only the Krylov state for vectors of 3 * n_vec entries (three
    // planes of n_vec); rhs is a device vector copied into the slot.
    int attach_vector(int s, void* mem, int64_t n_vec, int32_t k, const double* rhs);
    // beta = |rhs| and v_0.
    int start_vector(const std::vector<int>& slots);
    // The caller has written w = A P^{-1} v_j (desc.j) into desc.w: Gram-Schmidt,
    // Givens rotation and v_{j+1}; then the status rows are read back.
    int step_ortho(const std::vector<int>& slots);
    // step_ortho without reading the status rows back (see copy_status_async).
    int step_ortho_nowait(const std::vector<int>& slots);
    // For an iteration captured once into a HIP graph and replayed: ortho_lists sets and
    // uploads the Gram-Schmidt work lists of `slots` (fixed afterwards);
    // launch_ortho_fixed enqueues Gram-Schmidt, Givens and v_{j+1} on those lists on
    // stream s (the capturing stream), then advances each slot's iteration counter j on
    // the device, so a replay needs no upload.  dev_desc() is the device descriptor table (kernels of the caller read
    // the iteration's v_j through it).
    int ortho_lists(const std::vector<int>& slots);
    int launch_ortho_fixed(const std::vector<int>& slots, hipStream_t s);
    const SlotDesc* dev_desc() const { return dev_desc_; }
    // y from the least-squares problem and w = V_m y (iterations done in desc.j);
    // the caller forms x = P^{-1} w.
    int finalize_vector(const std::vector<int>& slots);
    const double* status(int s) const { return host_stat_ + NSTAT * s; }
    // Two pinned status rows ([MAX_SLOTS * NSTAT] each) and an event per row, for a
    // caller that reads the status of iteration j - 1 while iteration j runs.
    double* lag_row(int k);
    hipEvent_t lag_event(int k);
    SlotDesc& desc(int s) { return host_desc_[s]; }
    hipStream_t stream() const { return st_; }
    bool mixed() const { return mixed_; }

private:
    int upload();
    int launch_step(bool capture);
    int launch_ortho(bool capture, bool advance = false);
    void set_list(WL w, const std::vector<int>& slots);
    void set_sl_list(const std::vector<Part>& parts);
    int run_step();
    int read_status();

    int set_step_lists(const std::vector<Part>& parts);
    int launch_pre(const std::vector<int>& slots);
    int launch_red_ortho(const std::vector<int>& slots);
    int launch_or_replay();

    hipStream_t st_ = nullptr;
    bool mixed_ = false, doublet_ = true, use_graph_ = false;
    SlotDesc* host_desc_ = nullptr;   // [MAX_SLOTS], the host's current tables
    SlotDesc* dev_desc_ = nullptr;
    StepTables* host_tab_ = nullptr;
    StepTables* dev_tab_ = nullptr;
    // Uploads go through a ring of pinned snapshots of the tables, so the host may
    // change its tables for the next step while a copy of the last ones is in flight;
    // a stage is reused once the event recorded after its copy has completed.
    static constexpr int NSTAGE = UPLOAD_RING;
    struct Stage {
        SlotDesc* desc = nullptr;
        StepTables* tab = nullptr;
        hipEvent_t ev = nullptr;
        bool used = false;
    };
    Stage stage_[NSTAGE];
    int next_stage_ = 0;
    double* host_stat_ = nullptr;     // pinned [MAX_SLOTS * NSTAT]
    double* dev_stat_ = nullptr;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    BatchRes* res_ = nullptr;
};

}  // namespace stokes
