// Internal declarations shared by the translation units of libstokes.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "host_logic.hpp"
#include "stokes.h"

namespace stokes {

// ---- error reporting ------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define STOKES_HIP(call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #call);  \
    } while (0)

// ---- named ranges for the profiler's marker trace (roctx) -------------------
// One range per solver call or serving step, so a trace shows where each one's
// kernels begin and end; without a profiler attached a push or pop costs a call.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

// ---- kernel timing for measurement (stokes_profile_enable) -----------------
// prof_begin/prof_end bracket one launch of a main pair-sum kernel with HIP
// events on its stream when profiling is on; they do nothing otherwise.
void prof_begin(hipStream_t st);
void prof_end(hipStream_t st);

// ---- scratch workspace, one per (device, stream) -------------------------
// get() returns device memory of at least `bytes`, growing the buffer when
// needed (growing waits for `stream` so the old buffer is no longer in use).
struct Workspace {
    void* dev = nullptr;
    size_t bytes = 0;
    void* host = nullptr;      // small pinned host buffer for status read-back
};
int workspace_get(hipStream_t stream, size_t bytes, Workspace** out);
// Frees the implicit time step's cached device buffers (stokes_release_workspace).
void fiberstep_release();
// Frees the pinned tables, events and device tables that finished batched solves keep
// for the next one (stokes_release_workspace).
void batch_res_drain();

// The input scan of STOKES_CHECK_INPUTS for a single-layer sum's sources (synchronous on
// st): forces and weights finite, fiber ids in [0, n_fib) and non-decreasing, lengths
// finite.  E_NONFINITE or E_INVAL with `who` in the message; the workspace of st is used.
int scan_sl_inputs(hipStream_t st, const char* who, int64_t n_s, const double* force, const double* weight,
                   const int32_t* fib, int32_t n_fib, const double* flen);

// Slot option (beside STOKES_NONLOCAL and STOKES_PRECOND_BLOCK): the slot's single-layer
// sum is evaluated by the caller (a treecode) into partial row 0 instead of by k_sl.
constexpr uint32_t OPT_FAR = 1u << 20;

// Parameters of the solvers' treecode far field: degree 1..10, theta in (0, 1).
inline int check_far(const stokes_far* far, const char* who) {
    if (far && (far->degree < 1 || far->degree > 10 || !(far->theta > 0.0 && far->theta < 1.0)))
        return fail(STOKES_E_INVAL, std::string(who) + ": stokes_far needs degree 1..10 and theta in (0, 1)");
    return STOKES_OK;
}

// A treecode plan over fiber nodes (targets = sources) for the u_bar sums of the
// solvers; destroyed with the object.
struct FarPlan {
    stokes_tree* t = nullptr;
    FarPlan() = default;
    FarPlan(const FarPlan&) = delete;
    FarPlan& operator=(const FarPlan&) = delete;
    ~FarPlan() {
        if (t) (void)stokes_tree_destroy(t);
    }
    // Validates `far` and builds the plan (synchronous on st).
    int make(int64_t n, const double* xyz, const stokes_far& far, hipStream_t st);
};

struct Tile;
struct SrcDL64;
struct SrcDL32;

// A double-layer sum on a fixed geometry (sources, normals, weights, surface ids,
// targets and their self indices), evaluated for many densities: the tiles, the
// source packs and the exclusion ranges are made once, and an evaluation re-packs
// only the density.  The geometry arrays (device) must stay alive and unchanged
// while the plan is used; the plan owns its own device memory.  With surface ids
// (src_sid) the sources are several surfaces, and a target's own density is subtracted
// only from the sources of its own surface, the surface of its self source (always with
// the on-surface subtraction; the MULTI kernels).  Without, an evaluation gives the
// result of stokes_dl_eval with the same near radius and flags, bit for bit.
class DLPlan {
public:
    DLPlan() = default;
    ~DLPlan();
    DLPlan(const DLPlan&) = delete;
    DLPlan& operator=(const DLPlan&) = delete;
    int init(int64_t n_src, const double* src_xyz, const double* src_normal, const double* src_weight,
             const int32_t* src_sid, int64_t n_trg, const double* trg_xyz, const int64_t* trg_self,
             double near_r, uint32_t flags, hipStream_t st);
    // in_capture: the launch is being captured into a graph (no profiling events)
    int eval(const double* src_q, double* u_out, bool accumulate, hipStream_t st, bool in_capture = false);

private:
    void* mem_ = nullptr;
    bool mixed_ = false, sub_ = true, multi_ = false;
    int64_t n_s_ = 0, n_t_ = 0;
    const double* txyz_ = nullptr;
    float near2_ = 0.0f;
    Partition P_{};
    Tile* tiles_ = nullptr;
    SrcDL64* s64_ = nullptr;
    SrcDL32* s32_ = nullptr;
    int2* excl_ = nullptr;
    double* partial_ = nullptr;
};

// A tile of TILE consecutive sources with two bounding volumes: a sphere about
// the centre of its bounding box, and a capsule (a segment from the first to
// the last source plus a radius) that is much tighter for a straight fiber.
// A target that is outside either volume cannot meet an excluded, coincident
// or near pair in the tile.
struct __align__(16) Tile {
    double ox, oy, oz;   // FP64 origin: centre of the bounding box
    double reach2;       // FP64 path: a target closer than sqrt(reach2) may coincide with a source
    float reach2_f;      // mixed path: a target closer than this may have a near pair
    int32_t j0, j1;      // sources [j0, j1)
    float inv_l2;        // 1/|b|^2 of the capsule axis (0: the axis is a point)
    float ax, ay, az;    // capsule axis start, relative to the origin
    float bx, by, bz;    // capsule axis vector
    float cap2_f;        // mixed path: (capsule radius + near radius)^2, padded
    float cap2_d;        // FP64 path: (capsule radius)^2, padded
    float band2_f;       // mixed double layer: a target closer than this lies in the
                         // tile's tangent band (dl_band_radius); 0 otherwise
};

// Single-layer source, premultiplied: s = w f / (8 pi mu), c = (eps L)^2/2, c3 = -3 c.
struct __align__(64) SrcSL64 { double x, y, z, c, sx, sy, sz, c3; };
// Same in FP32 with tile-local coordinates (position minus the tile origin).
struct __align__(32) SrcSL32 { float x, y, z, c, sx, sy, sz, c3; };
// Double-layer source: n' = (3/(4 pi)) w n.
struct __align__(32) SrcDL64 { double x, y, z, qx, qy, qz, nx, ny, nz, pad0, pad1, pad2; };
struct __align__(16) SrcDL32 { float x, y, z, qx, qy, qz, nx, ny, nz, pad0, pad1, pad2; };

}  // namespace stokes
