// Internal declarations shared by the translation units of libstokes.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

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
// Double layer over several surfaces in one sum: src_sid gives each source's surface;
// a target's own density is subtracted only from its own surface's sources (the
// surface of its self source).  Always with the on-surface subtraction.
int dl_eval_surfaces(int64_t n_src, const double* src_xyz, const double* src_normal, const double* src_weight,
                     const double* src_q, const int32_t* src_sid, int64_t n_trg, const double* trg_xyz,
                     const int64_t* trg_self, double near_r, uint32_t flags, double* u_out, hipStream_t st);

// Bump allocator over a workspace buffer (256-byte aligned slices).
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + off);
        off += n * sizeof(T);
        return p;
    }
    static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
};

// ---- geometry of the kernel sums -----------------------------------------
constexpr int TILE = 32;      // sources per tile (one 32-node fiber in the benchmark geometries)
constexpr int BLOCK = 256;    // 4 waves per block
// Targets per lane (register blocking) of each pair kernel, and the number of
// blocks a launch aims for (many small work items keep all 256 CUs busy to
// the end; measured on gfx950: R = 1 with ~64k blocks is fastest for both
// precisions, because occupancy matters more here than reuse of the SGPR
// source operands).
constexpr int R_SL64 = 1, R_SL32 = 1, R_DL64 = 1, R_DL32 = 1;
constexpr int64_t TARGET_BLOCKS = 65536;
// Serving slots share the GPU with other requests, so each uses fewer chunks
// (less partial-sum memory per request).
constexpr int64_t TARGET_BLOCKS_SLOT = 4096;
constexpr int MIN_TILES_PER_CHUNK = 8;

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
};

// Single-layer source, premultiplied: s = w f / (8 pi mu), c = (eps L)^2/2, c3 = -3 c.
struct __align__(64) SrcSL64 { double x, y, z, c, sx, sy, sz, c3; };
// Same in FP32 with tile-local coordinates (position minus the tile origin).
struct __align__(32) SrcSL32 { float x, y, z, c, sx, sy, sz, c3; };
// Double-layer source: n' = (3/(4 pi)) w n.
struct __align__(32) SrcDL64 { double x, y, z, qx, qy, qz, nx, ny, nz, pad0, pad1, pad2; };
struct __align__(16) SrcDL32 { float x, y, z, qx, qy, qz, nx, ny, nz, pad0, pad1, pad2; };

// Work partition of one sum: targets in waves of 64*R, sources in chunks of
// whole tiles.  Depends only on the problem sizes (bitwise reproducibility).
struct Partition {
    int R;
    int64_t n_t;
    int32_t n_tiles;
    int32_t tiles_per_chunk;
    int32_t n_chunks;
    int32_t n_tblocks;
};
// min_tiles_small: least source tiles per chunk when there are fewer than 64
// target blocks (a problem too small to fill the chip with target blocks alone).
Partition make_partition(int64_t n_t, int64_t n_s, int R, int64_t target_blocks = TARGET_BLOCKS,
                         int min_tiles_small = 1);

}  // namespace stokes
