// Kernel sums of the free-space Stokes fundamental solutions on gfx950.
//
// Single layer (Stokeslet + doublet, eq. oseen and eq. main-sb-vel) and
// double layer (stresslet, eq. stresslet / eq. double-layer, with the
// on-surface singularity subtraction) as direct O(N M) sums.
//
// Execution scheme (all kernels are VALU-bound; there is no dense
// contraction here, so no MFMA):
//   * targets: each lane owns R targets (register blocking), a wave 64 R
//     consecutive targets, a block 4 waves;
//   * sources: grouped in tiles of TILE = 32 consecutive points (one fiber of
//     32 nodes, or a compact 4 x 8 patch of the sphere grid) and in chunks of
//     whole tiles; the grid is (target blocks) x (source chunks), and each
//     chunk writes an FP64 partial that a second kernel adds in chunk order,
//     so results are bitwise reproducible;
//   * every lane of a wave walks the same source, so sources are read with
//     wave-uniform addresses: the compiler turns them into scalar loads and
//     the pair arithmetic takes them straight from SGPRs (the broadcast costs
//     no vector instruction and no LDS traffic);
//   * per (wave, tile) a bounding-sphere test decides whether any lane may
//     meet an excluded, coincident or (mixed path) near pair in the tile; if
//     none can, the tile runs a branch-free loop, otherwise a checked loop.
//
// Mixed path: coordinates are rounded to FP32 relative to the tile origin
// (target: fl32(x - o) computed in FP64 once per tile; source: fl32(y - o)),
// so the FP32 difference d keeps relative accuracy ~ 2^-24 (1 + tile
// radius / |d|).  Pairs with FP32 |d|^2 below the source's near threshold are
// masked out of the FP32 loop and recomputed in FP64 from the FP64 inputs;
// the same FP32 test decides both, so every pair is counted exactly once.
// The FP32 tile partial is added to a Kahan-compensated FP32 pair (S, C) per
// target component; chunk partials are FP64.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "stokes_internal.hpp"
#include "sum_device.hpp"

namespace stokes {

// ---- preparation kernels -------------------------------------------------------

// Tile bounds take 32 lanes per tile (tile_prep_half), TILE_PREP_BLOCK threads per block.
// near_r: extra reach for the mixed path; the per-source near radius is max(near_r,
// near_fac * L_fiber) when flen/sfib are given.  band < 0 (mixed double layer): each
// tile's tangent band from the normals nrm.
constexpr int TILE_PREP_BLOCK = 256;
static inline unsigned tile_prep_blocks(int64_t n_tiles) {
    return (unsigned)((n_tiles * 32 + TILE_PREP_BLOCK - 1) / TILE_PREP_BLOCK);
}

// The set-up of a sum in one launch.  Blocks below tile_blocks take whole tiles, a
// half-wave each: tile_prep_half, then lane l packs the tile's source t TILE + l
// against the tile's FP64 origin (single layer, or double layer when DL).  The other
// blocks write the self-exclusion range of target i (n_t = 0: none).
struct PrepArgs {
    int64_t n_s;
    const double* sx;
    int32_t n_tiles;
    unsigned tile_blocks;
    double near_r, near_fac, band;       // tile_prep_half
    const int32_t* sfib;
    int32_t n_fib;
    const double* flen;
    const double* nrm;                   // double layer: normals (also the band's)
    Tile* tiles;
    const double* f;                     // single layer: forces; double layer: density
    const double* w;
    double pref, eps, src_near_r;        // single layer
    int doublet;
    const int32_t* sid;                  // double layer: surface ids or null
    void* s64;
    void* s32;
    float* near_t;
    int64_t n_t;                         // self exclusion
    const int64_t* tself;
    int identity;
    int2* excl;
    unsigned long long* counters;
};

template <bool DL>
__global__ __launch_bounds__(TILE_PREP_BLOCK) void prep_kernel(PrepArgs p) {
    if (blockIdx.x < p.tile_blocks) {
        const int t = (int)((blockIdx.x * TILE_PREP_BLOCK + threadIdx.x) / 32);
        const int l = threadIdx.x & 31;
        if (t >= p.n_tiles) return;   // whole half-waves
        const Tile T = tile_prep_half(t, l, p.n_s, p.sx, p.near_r, p.near_fac, p.sfib, p.n_fib, p.flen,
                                      p.tiles, p.band, p.nrm);
        const int64_t j = (int64_t)t * TILE + l;
        if (j >= p.n_s) return;
        if (DL)
            dl_src_pack(j, p.n_s, p.sx, p.nrm, p.w, p.f, p.sid, T.ox, T.oy, T.oz, static_cast<SrcDL64*>(p.s64),
                        static_cast<SrcDL32*>(p.s32));
        else
            sl_src_pack(j, p.n_s, p.sx, p.f, p.w, p.sfib, p.n_fib, p.flen, p.pref, p.eps, p.doublet,
                        p.src_near_r, T.ox, T.oy, T.oz, static_cast<SrcSL64*>(p.s64),
                        static_cast<SrcSL32*>(p.s32), p.near_t);
        return;
    }
    const int64_t i = (int64_t)(blockIdx.x - p.tile_blocks) * TILE_PREP_BLOCK + threadIdx.x;
    unsigned long long cnt = 0;
    if (i < p.n_t) {
        const int64_t s = p.tself ? p.tself[i] : (p.identity ? i : -1);
        int2 e = make_int2(0, 0);
        if (s >= 0 && s < p.n_s) {
            e = make_int2((int)s, (int)s + 1);
            cnt = 1;
        }
        p.excl[i] = e;
    }
    if (p.counters) wave_count(p.counters + 2, cnt);
}

static unsigned prep_grid(const PrepArgs& p) {
    return p.tile_blocks + (unsigned)((p.n_t + TILE_PREP_BLOCK - 1) / TILE_PREP_BLOCK);
}

__global__ void fill_int2_kernel(int2* p, int64_t n, int2 v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Start/end source index of every fiber (fiber ids non-decreasing).
__global__ void fiber_bounds_kernel(int64_t n_s, const int32_t* __restrict__ sfib, int32_t n_fib,
                                    int2* bounds) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_s) return;
    const int f = sfib[j];
    if (f < 0 || f >= n_fib) return;
    if (j == 0 || sfib[j - 1] != f) bounds[f].x = (int)j;
    if (j == n_s - 1 || sfib[j + 1] != f) bounds[f].y = (int)(j + 1);
}

__global__ void excl_fiber_kernel(int64_t n_t, const int32_t* __restrict__ tfib,
                                  const int2* __restrict__ bounds, int32_t n_fib, int2* excl,
                                  unsigned long long* counters) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long cnt = 0;
    if (i < n_t) {
        const int f = tfib[i];
        int2 e = make_int2(0, 0);
        if (f >= 0 && f < n_fib) {
            e = bounds[f];
            if (e.y < e.x) e = make_int2(0, 0);
        }
        excl[i] = e;
        cnt = (unsigned long long)(e.y - e.x);
    }
    if (counters) wave_count(counters + 2, cnt);
}

// out = (accumulate ? out : 0) + sum_k partial[k]  (+ jump term), chunk order fixed.
// Sum of the chunk partials per target (plus the double layer's jump term).  A
// workgroup takes 64 targets with eight threads each: thread slice sl sums chunks
// sl, sl + 8, ... in order (four chunks' loads issued before their adds, so that a
// thread has twelve loads in flight), and the eight slice sums are added in a fixed
// order, so the result does not depend on the launch.
constexpr int RED_T = 64, RED_S = 8;
__global__ __launch_bounds__(RED_T * RED_S) void reduce_kernel(int64_t n_t, int32_t n_chunks,
                                                              const double* __restrict__ partial,
                                                              int accumulate, double* out, int64_t out_stride,
                                                              const int2* __restrict__ excl,
                                                              const double* __restrict__ q, int64_t n_s,
                                                              double jump, int round_q = 0) {
    __shared__ double part[RED_S - 1][3][RED_T];
    const int tx = threadIdx.x % RED_T, sl = threadIdx.x / RED_T;
    const int64_t i = (int64_t)blockIdx.x * RED_T + tx;
    double v[3] = {0.0, 0.0, 0.0};
    if (i < n_t) {
        int k = sl;
        for (; k + 3 * RED_S < n_chunks; k += 4 * RED_S) {
            double a[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double* p = partial + (int64_t)(k + u * RED_S) * 3 * n_t;
                a[u][0] = p[i];
                a[u][1] = p[n_t + i];
                a[u][2] = p[2 * n_t + i];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                for (int c = 0; c < 3; ++c) v[c] += a[u][c];
        }
        for (; k < n_chunks; k += RED_S) {
            const double* p = partial + (int64_t)k * 3 * n_t;
            v[0] += p[i];
            v[1] += p[n_t + i];
            v[2] += p[2 * n_t + i];
        }
    }
    if (sl > 0)
        for (int c = 0; c < 3; ++c) part[sl - 1][c][tx] = v[c];
    __syncthreads();
    if (sl > 0 || i >= n_t) return;
    for (int s2 = 0; s2 < RED_S - 1; ++s2)
        for (int c = 0; c < 3; ++c) v[c] += part[s2][c][tx];
    if (q && excl) {
        const int2 e = excl[i];
        if (e.y > e.x) {
            // round_q: the sum subtracted fl32(q_self) (dl_mixed_wave), so the jump takes it too
            double qs[3] = {q[e.x], q[n_s + e.x], q[2 * n_s + e.x]};
            if (round_q)
                for (int c = 0; c < 3; ++c) qs[c] = (double)(float)qs[c];
            v[0] += jump * qs[0];
            v[1] += jump * qs[1];
            v[2] += jump * qs[2];
        }
    }
    for (int c = 0; c < 3; ++c) {
        double* o = out + c * out_stride + i;
        *o = accumulate ? *o + v[c] : v[c];
    }
}

inline unsigned red_blocks(int64_t n_t) { return (unsigned)((n_t + RED_T - 1) / RED_T); }

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// Non-finite / range scan; sets bits in *flag (1 = non-finite, 2 = bad fiber ids).
__global__ void check_finite_kernel(const double* __restrict__ p, int64_t n, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(p[i])) atomicOr(flag, 1);
}
__global__ void check_fiber_kernel(const int32_t* __restrict__ fib, int64_t n, int32_t n_fib,
                                   int* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int f = fib[i];
    bool bad = (f < 0 || f >= n_fib);
    if (i > 0 && fib[i - 1] > f) bad = true;
    if (bad) atomicOr(flag, 2);
}

// ---- host side -----------------------------------------------------------------

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }


// Scratch layout of one sum (both layers use the same carve order).
struct SumScratch {
    Tile* tiles;
    void* s64;
    void* s32;
    float* near_t;
    int2* excl;
    int2* fbounds;
    double* partial;
    unsigned long long* counters;
    int* flag;
};

static size_t sum_scratch_bytes(int64_t n_s, int64_t n_t, int32_t n_fib, size_t s64b, size_t s32b,
                                int32_t n_chunks) {
    return sum_layout(n_s, n_t, n_fib, sizeof(Tile), s64b, s32b, n_chunks).bytes;
}

static SumScratch carve_sum(void* base, int64_t n_s, int64_t n_t, int32_t n_fib, size_t s64b,
                            size_t s32b, int32_t n_chunks) {
    const SumLayout L = sum_layout(n_s, n_t, n_fib, sizeof(Tile), s64b, s32b, n_chunks);
    char* b = static_cast<char*>(base);
    SumScratch s;
    s.tiles = reinterpret_cast<Tile*>(b + L.tiles);
    s.s64 = b + L.s64;
    s.s32 = s32b ? b + L.s32 : nullptr;
    s.near_t = reinterpret_cast<float*>(b + L.near_t);
    s.excl = reinterpret_cast<int2*>(b + L.excl);
    s.fbounds = reinterpret_cast<int2*>(b + L.fbounds);
    s.partial = reinterpret_cast<double*>(b + L.partial);
    s.counters = reinterpret_cast<unsigned long long*>(b + L.counters);
    s.flag = reinterpret_cast<int*>(b + L.flag);
    return s;
}

// The launch of a pair kernel has P.grid() workgroups; workgroup g writes chunk
// g / n_tblocks of the partials, which hold P.n_chunks rows of 3 n_t.  Checked on the
// host before every launch (a grid that outgrew its partial buffer would write past it).
static int check_grid(const Partition& P, unsigned grid, int64_t n_t) {
    if ((int64_t)grid != P.grid() || P.n_t != n_t || P.grid() > INT32_MAX ||
        (int64_t)P.n_chunks * P.tiles_per_chunk < P.n_tiles ||
        (P.n_chunks > 0 && (int64_t)(P.n_chunks - 1) * P.tiles_per_chunk >= P.n_tiles))
        return fail(STOKES_E_INVAL, "internal: launch grid does not match the sum's partition");
    return STOKES_OK;
}

// The register blocking R must match the one the partition was made with.
static void launch_sl_kernel(bool mixed, bool doublet, unsigned grid, const SumArgs& a,
                             hipStream_t st) {
    if (mixed) {
        if (doublet)
            hipLaunchKernelGGL((sl_mixed_kernel<R_SL32, true>), dim3(grid), dim3(BLOCK), 0, st, a);
        else
            hipLaunchKernelGGL((sl_mixed_kernel<R_SL32, false>), dim3(grid), dim3(BLOCK), 0, st, a);
    } else {
        if (doublet)
            hipLaunchKernelGGL((sl_fp64_kernel<R_SL64, true>), dim3(grid), dim3(BLOCK), 0, st, a);
        else
            hipLaunchKernelGGL((sl_fp64_kernel<R_SL64, false>), dim3(grid), dim3(BLOCK), 0, st, a);
    }
}

// Core launcher: exclusion ranges must already be in `excl` (or null).
// One single-layer problem, with the targets resolved (never null here).
struct SLProblem {
    int64_t n_s;
    const double* sxyz;
    const double* force;
    const double* weight;      // may be null
    const int32_t* sfib;       // may be null
    int32_t n_fib;
    const double* flen;        // may be null
    int64_t n_t;
    const double* txyz;
    int64_t t_stride;
    double mu, eps, near_r;
    bool mixed, doublet, accumulate;
    double* u;                 // [3][n_t], stride n_t
};

// Start/end source index of every fiber (fiber ids non-decreasing).
static int fiber_bounds_launch(int64_t n_s, const int32_t* sfib, int32_t n_fib, int2* bounds,
                               hipStream_t st) {
    if (n_fib > 0)
        hipLaunchKernelGGL(fill_int2_kernel, dim3(nblk(n_fib)), dim3(256), 0, st, bounds,
                           (int64_t)n_fib, make_int2(0, 0));
    if (n_s > 0)
        hipLaunchKernelGGL(fiber_bounds_kernel, dim3(nblk(n_s)), dim3(256), 0, st, n_s, sfib, n_fib,
                           bounds);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

// self_excl: the exclusion ranges come from self indices (tself, or the identity) and
// are written by the set-up launch; otherwise excl was made before (or is null).
static int sl_core(const SLProblem& p, const Partition& P, const SumScratch& S, const int2* excl,
                   bool self_excl, const int64_t* tself, int identity, unsigned long long* counters,
                   hipStream_t st) {
    if (P.n_chunks > 0) {
        PrepArgs q{};
        q.n_s = p.n_s;
        q.sx = p.sxyz;
        q.n_tiles = P.n_tiles;
        q.tile_blocks = tile_prep_blocks(P.n_tiles);
        q.near_r = p.mixed ? std::max(p.near_r, 0.0) : 0.0;
        q.near_fac = p.mixed ? 2.0 * p.eps : 0.0;
        q.band = 0.0;
        q.sfib = p.sfib;
        q.n_fib = p.n_fib;
        q.flen = p.flen;
        q.tiles = S.tiles;
        q.f = p.force;
        q.w = p.weight;
        q.pref = 1.0 / (8.0 * PI_D * p.mu);
        q.eps = p.eps;
        q.src_near_r = std::max(p.near_r, 0.0);
        q.doublet = p.doublet ? 1 : 0;
        q.s64 = S.s64;
        q.s32 = p.mixed ? S.s32 : nullptr;
        q.near_t = S.near_t;
        if (self_excl) {
            q.n_t = p.n_t;
            q.tself = tself;
            q.identity = identity;
            q.excl = S.excl;
            q.counters = counters;
        }
        hipLaunchKernelGGL(prep_kernel<false>, dim3(prep_grid(q)), dim3(TILE_PREP_BLOCK), 0, st, q);
        SumArgs a{};
        a.tx = p.txyz;
        a.t_stride = p.t_stride;
        a.n_t = p.n_t;
        a.excl = excl;
        a.tiles = S.tiles;
        a.n_tiles = P.n_tiles;
        a.tiles_per_chunk = P.tiles_per_chunk;
        a.n_tblocks = P.n_tblocks;
        a.s64 = S.s64;
        a.s32 = S.s32;
        a.near_t = S.near_t;
        a.n_s = p.n_s;
        a.partial = S.partial;
        a.counters = counters;
        const unsigned grid = (unsigned)((int64_t)P.n_tblocks * P.n_chunks);
        if (int rc = check_grid(P, grid, p.n_t)) return rc;
        prof_begin(st);
        launch_sl_kernel(p.mixed, p.doublet, grid, a, st);
        prof_end(st);
        STOKES_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(reduce_kernel, dim3(red_blocks(p.n_t)), dim3(RED_T * RED_S), 0, st, p.n_t, P.n_chunks,
                       S.partial, p.accumulate ? 1 : 0, p.u, p.n_t, (const int2*)nullptr,
                       (const double*)nullptr, (int64_t)0, 0.0);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}




// ---- validation helpers ---------------------------------------------------------
static bool bad_ptr(const void* p, int64_t n) { return p == nullptr && n > 0; }

struct Check {
    int* flag;
    hipStream_t st;
    void finite(const double* p, int64_t n) {
        if (p && n > 0)
            hipLaunchKernelGGL(check_finite_kernel, dim3(nblk(n)), dim3(256), 0, st, p, n, flag);
    }
    void fiber(const int32_t* p, int64_t n, int32_t n_fib) {
        if (p && n > 0)
            hipLaunchKernelGGL(check_fiber_kernel, dim3(nblk(n)), dim3(256), 0, st, p, n, n_fib,
                               flag);
    }
};

static int read_flag(Workspace* ws, int* flag, hipStream_t st, int* out) {
    STOKES_HIP(hipMemcpyAsync(ws->host, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    STOKES_HIP(hipStreamSynchronize(st));
    *out = *static_cast<int*>(ws->host);
    return STOKES_OK;
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

int scan_sl_inputs(hipStream_t st, const char* who, int64_t n_s, const double* force, const double* weight,
                   const int32_t* fib, int32_t n_fib, const double* flen) {
    Workspace* ws = nullptr;
    if (int rc = workspace_get(st, 256, &ws)) return rc;
    int* flag = static_cast<int*>(ws->dev);
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, flag);
    Check c{flag, st};
    c.finite(force, 3 * n_s);
    c.finite(weight, n_s);
    c.finite(flen, fib ? n_fib : 0);
    c.fiber(fib, n_s, n_fib);
    STOKES_HIP(hipGetLastError());
    int f = 0;
    if (int rc = read_flag(ws, flag, st, &f)) return rc;
    if (f & 2) return fail(STOKES_E_INVAL, std::string(who) + ": fiber ids out of range or decreasing");
    if (f & 1) return fail(STOKES_E_NONFINITE, std::string(who) + ": non-finite input");
    return STOKES_OK;
}

static int finish_diag(Workspace* ws, unsigned long long* counters, hipStream_t st, int64_t n_t,
                       int64_t n_s, stokes_diag* diag) {
    STOKES_HIP(hipMemcpyAsync(ws->host, counters, 3 * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, st));
    STOKES_HIP(hipStreamSynchronize(st));
    const unsigned long long* h = static_cast<const unsigned long long*>(ws->host);
    diag->near_pairs = (int64_t)h[0];
    diag->coincident = (int64_t)h[1];
    diag->pairs = n_t * n_s - (int64_t)h[2] - (int64_t)h[1];
    return STOKES_OK;
}

}  // namespace stokes

using namespace stokes;

// Scratch of the entry point that allocates nothing (stokes_sl_eval_noalloc): one
// array per GPU, in the library's device code object, held until the process ends.
// Host code reaches it only through the address hipGetSymbolAddress returns for the
// current device (the array's name is not a device address on the host).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` on the current device, resolved once per device.
static int noalloc_scratch(void** out) {
    static std::mutex mu;
    static void* addr[64] = {};
    int dev = 0;
    STOKES_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(STOKES_E_INVAL, "stokes_sl_eval_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(STOKES_E_DEVICE, "stokes_sl_eval_noalloc: no device address for the scratch array");
        addr[dev] = p;
    }
    *out = addr[dev];
    return STOKES_OK;
}

// fixed: the call's scratch is `fixed` (fixed_cap bytes) instead of the library's
// workspace, and nothing is allocated; the partition then takes fewer source chunks
// when the standard one's partials do not fit (the reduction order, and so the last
// bits of the result, follow the partition).
static int sl_run(int64_t n_src, const double* src_xyz, const double* src_force,
                  const double* src_weight, const int32_t* src_fiber, int32_t n_fib,
                  const double* fiber_len, int64_t n_trg, const double* trg_xyz,
                  const int64_t* trg_self, const int32_t* trg_fiber, double mu,
                  double eps, double near_r, uint32_t flags, double* u_out,
                  void* stream, stokes_diag* diag, bool noalloc) {
    uint32_t known = STOKES_PREC_MIXED | STOKES_EXCL_SELF_POINT | STOKES_EXCL_SAME_FIBER |
                     STOKES_NO_DOUBLET | STOKES_ACCUMULATE | STOKES_CHECK_INPUTS;
    if (noalloc) known &= ~(uint32_t)STOKES_CHECK_INPUTS;   // its read-back needs a host buffer
    if (flags & ~known) return fail(STOKES_E_INVAL, "stokes_sl_eval: unknown flag bits");
    const bool self_mode = flags & STOKES_EXCL_SELF_POINT;
    const bool fiber_mode = flags & STOKES_EXCL_SAME_FIBER;
    if (self_mode && fiber_mode)
        return fail(STOKES_E_INVAL, "stokes_sl_eval: choose one exclusion mode");
    if (n_src < 0) return fail(STOKES_E_INVAL, "stokes_sl_eval: n_src < 0");
    const bool same = (trg_xyz == nullptr);
    const int64_t n_t = same ? n_src : n_trg;
    if (n_t < 0) return fail(STOKES_E_INVAL, "stokes_sl_eval: n_trg < 0");
    if (n_src >= (int64_t)1 << 31 || n_t >= (int64_t)1 << 31)
        return fail(STOKES_E_INVAL, "stokes_sl_eval: more than 2^31-1 sources or targets");
    if (bad_ptr(src_xyz, n_src) || bad_ptr(src_force, n_src))
        return fail(STOKES_E_INVAL, "stokes_sl_eval: null source array");
    if (bad_ptr(u_out, n_t)) return fail(STOKES_E_INVAL, "stokes_sl_eval: null u_out");
    if (!(mu > 0.0) || !std::isfinite(mu)) return fail(STOKES_E_INVAL, "stokes_sl_eval: mu must be > 0");
    if (!(eps > 0.0 && eps < 0.5)) return fail(STOKES_E_INVAL, "stokes_sl_eval: eps must be in (0, 0.5)");
    if (!std::isfinite(near_r)) return fail(STOKES_E_INVAL, "stokes_sl_eval: near_r not finite");
    if (n_fib < 0) return fail(STOKES_E_INVAL, "stokes_sl_eval: n_fib < 0");
    if (src_fiber && n_fib == 0 && n_src > 0)
        return fail(STOKES_E_INVAL, "stokes_sl_eval: src_fiber given with n_fib = 0");
    if (fiber_mode && (src_fiber == nullptr && n_src > 0))
        return fail(STOKES_E_INVAL, "stokes_sl_eval: STOKES_EXCL_SAME_FIBER needs src_fiber");
    if (fiber_mode && !same && trg_fiber == nullptr && n_t > 0)
        return fail(STOKES_E_INVAL, "stokes_sl_eval: STOKES_EXCL_SAME_FIBER needs trg_fiber");
    if (n_t == 0) {
        if (diag) *diag = stokes_diag{0, 0, 0};
        return STOKES_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool mixed = flags & STOKES_PREC_MIXED;
    Partition P = make_partition(n_t, n_src, mixed ? R_SL32 : R_SL64);
    const int32_t nf = src_fiber ? n_fib : 0;
    const size_t s32b = mixed ? sizeof(SrcSL32) : 0;
    Workspace* ws = nullptr;
    void* base = nullptr;
    int rc = STOKES_OK;
    if (noalloc) {
        // the most source chunks (up to the standard partition's) whose partials fit
        auto bytes = [&](const Partition& Q) {
            return sum_scratch_bytes(n_src, n_t, nf, sizeof(SrcSL64), s32b, Q.n_chunks);
        };
        if (bytes(P) > NOALLOC_SCRATCH_BYTES) {
            int64_t lo = P.n_tblocks, hi = (int64_t)P.n_tblocks * std::max(P.n_chunks, 1);
            Partition best = make_partition(n_t, n_src, P.R, lo);
            if (bytes(best) > NOALLOC_SCRATCH_BYTES)
                return fail(STOKES_E_INVAL, "stokes_sl_eval_noalloc: " + std::to_string(n_src) + " sources and " +
                                                std::to_string(n_t) + " targets need more than the " +
                                                std::to_string(NOALLOC_SCRATCH_BYTES >> 20) +
                                                " MiB static scratch");
            while (lo < hi) {   // largest target_blocks that still fits
                const int64_t mid = lo + (hi - lo + 1) / 2;
                const Partition Q = make_partition(n_t, n_src, P.R, mid);
                if (bytes(Q) <= NOALLOC_SCRATCH_BYTES) {
                    lo = mid;
                    best = Q;
                } else {
                    hi = mid - 1;
                }
            }
            P = best;
        }
        if ((rc = noalloc_scratch(&base))) return rc;
    } else {
        rc = workspace_get(st, sum_scratch_bytes(n_src, n_t, nf, sizeof(SrcSL64), s32b, P.n_chunks), &ws);
        if (rc) return rc;
        base = ws->dev;
    }
    const SumScratch S = carve_sum(base, n_src, n_t, nf, sizeof(SrcSL64), s32b, P.n_chunks);
    if (flags & STOKES_CHECK_INPUTS) {
        hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, S.flag);
        Check c{S.flag, st};
        c.finite(src_xyz, 3 * n_src);
        c.finite(src_force, 3 * n_src);
        c.finite(src_weight, n_src);
        c.finite(fiber_len, nf);
        if (!same) c.finite(trg_xyz, 3 * n_t);
        c.fiber(src_fiber, n_src, n_fib);
        STOKES_HIP(hipGetLastError());
        int f = 0;
        if ((rc = read_flag(ws, S.flag, st, &f))) return rc;
        if (f & 2) return fail(STOKES_E_INVAL, "stokes_sl_eval: fiber ids out of range or decreasing");
        if (f & 1) return fail(STOKES_E_NONFINITE, "stokes_sl_eval: non-finite input");
    }
    unsigned long long* counters = diag ? S.counters : nullptr;
    if (counters) hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, counters, 4);
    const int2* excl = nullptr;
    const bool self_excl = self_mode && (trg_self || same);   // made in sl_core's set-up launch
    if (self_excl) {
        excl = S.excl;
    } else if (fiber_mode && n_src > 0) {
        if ((rc = fiber_bounds_launch(n_src, src_fiber, n_fib, S.fbounds, st))) return rc;
        const int32_t* tf = trg_fiber ? trg_fiber : src_fiber;
        hipLaunchKernelGGL(excl_fiber_kernel, dim3(nblk(n_t)), dim3(256), 0, st, n_t, tf,
                           S.fbounds, n_fib, S.excl, counters);
        excl = S.excl;
    }
    STOKES_HIP(hipGetLastError());
    SLProblem p{};
    p.n_s = n_src;
    p.sxyz = src_xyz;
    p.force = src_force;
    p.weight = src_weight;
    p.sfib = src_fiber;
    p.n_fib = nf;
    p.flen = fiber_len;
    p.n_t = n_t;
    p.txyz = same ? src_xyz : trg_xyz;
    p.t_stride = same ? n_src : n_t;
    p.mu = mu;
    p.eps = eps;
    p.near_r = near_r;
    p.mixed = mixed;
    p.doublet = !(flags & STOKES_NO_DOUBLET);
    p.accumulate = flags & STOKES_ACCUMULATE;
    p.u = u_out;
    if ((rc = sl_core(p, P, S, excl, self_excl, trg_self, same ? 1 : 0, counters, st))) return rc;
    if (diag) return finish_diag(ws, counters, st, n_t, n_src, diag);
    return STOKES_OK;
}

extern "C" int stokes_sl_eval(int64_t n_src, const double* src_xyz, const double* src_force,
                              const double* src_weight, const int32_t* src_fiber, int32_t n_fib,
                              const double* fiber_len, int64_t n_trg, const double* trg_xyz,
                              const int64_t* trg_self, const int32_t* trg_fiber, double mu,
                              double eps, double near_r, uint32_t flags, double* u_out,
                              void* stream, stokes_diag* diag) {
    return sl_run(n_src, src_xyz, src_force, src_weight, src_fiber, n_fib, fiber_len, n_trg, trg_xyz, trg_self,
                  trg_fiber, mu, eps, near_r, flags, u_out, stream, diag, false);
}

extern "C" int stokes_sl_eval_noalloc(int64_t n_src, const double* src_xyz, const double* src_force,
                                      const double* src_weight, const int32_t* src_fiber, int32_t n_fib,
                                      const double* fiber_len, int64_t n_trg, const double* trg_xyz,
                                      const int64_t* trg_self, const int32_t* trg_fiber, double mu,
                                      double eps, double near_r, uint32_t flags, double* u_out,
                                      void* stream) {
    return sl_run(n_src, src_xyz, src_force, src_weight, src_fiber, n_fib, fiber_len, n_trg, trg_xyz, trg_self,
                  trg_fiber, mu, eps, near_r, flags, u_out, stream, nullptr, true);
}

static void launch_dl_kernel(bool mixed, bool sub, bool multi, unsigned grid, const SumArgs& a,
                             hipStream_t st) {
    if (multi) {   // (always with the on-surface subtraction)
        if (mixed)
            hipLaunchKernelGGL((dl_mixed_kernel<R_DL32, true, true>), dim3(grid), dim3(BLOCK), 0, st, a);
        else
            hipLaunchKernelGGL((dl_fp64_kernel<R_DL64, true, true>), dim3(grid), dim3(BLOCK), 0, st, a);
        return;
    }
    if (mixed) {
        if (sub)
            hipLaunchKernelGGL((dl_mixed_kernel<R_DL32, true>), dim3(grid), dim3(BLOCK), 0, st, a);
        else
            hipLaunchKernelGGL((dl_mixed_kernel<R_DL32, false>), dim3(grid), dim3(BLOCK), 0, st, a);
    } else {
        if (sub)
            hipLaunchKernelGGL((dl_fp64_kernel<R_DL64, true>), dim3(grid), dim3(BLOCK), 0, st, a);
        else
            hipLaunchKernelGGL((dl_fp64_kernel<R_DL64, false>), dim3(grid), dim3(BLOCK), 0, st, a);
    }
}

static int dl_run(int64_t n_src, const double* src_xyz, const double* src_normal,
                  const double* src_weight, const double* src_q, const int32_t* src_sid, int64_t n_trg,
                  const double* trg_xyz, const int64_t* trg_self, double near_r, uint32_t flags,
                  double* u_out, void* stream, stokes_diag* diag) {
    const uint32_t known = STOKES_PREC_MIXED | STOKES_ONSURF_RAW | STOKES_ACCUMULATE |
                           STOKES_CHECK_INPUTS;
    if (flags & ~known) return fail(STOKES_E_INVAL, "stokes_dl_eval: unknown flag bits");
    if (n_src < 0) return fail(STOKES_E_INVAL, "stokes_dl_eval: n_src < 0");
    const bool same = (trg_xyz == nullptr);
    const int64_t n_t = same ? n_src : n_trg;
    if (n_t < 0) return fail(STOKES_E_INVAL, "stokes_dl_eval: n_trg < 0");
    if (n_src >= (int64_t)1 << 31 || n_t >= (int64_t)1 << 31)
        return fail(STOKES_E_INVAL, "stokes_dl_eval: more than 2^31-1 sources or targets");
    if (bad_ptr(src_xyz, n_src) || bad_ptr(src_normal, n_src) || bad_ptr(src_weight, n_src) ||
        bad_ptr(src_q, n_src))
        return fail(STOKES_E_INVAL, "stokes_dl_eval: null source array");
    if (bad_ptr(u_out, n_t)) return fail(STOKES_E_INVAL, "stokes_dl_eval: null u_out");
    if (!std::isfinite(near_r)) return fail(STOKES_E_INVAL, "stokes_dl_eval: near_r not finite");
    if (n_t == 0) {
        if (diag) *diag = stokes_diag{0, 0, 0};
        return STOKES_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool mixed = flags & STOKES_PREC_MIXED;
    const bool sub = !(flags & STOKES_ONSURF_RAW);
    const double nr = near_r > 0.0 ? near_r : 0.02;
    const Partition P = make_partition(n_t, n_src, mixed ? R_DL32 : R_DL64, TARGET_BLOCKS, 1, MIN_TILES_PER_CHUNK_DL);
    Workspace* ws = nullptr;
    int rc = workspace_get(st, sum_scratch_bytes(n_src, n_t, 0, sizeof(SrcDL64),
                                                 mixed ? sizeof(SrcDL32) : 0, P.n_chunks), &ws);
    if (rc) return rc;
    const SumScratch S = carve_sum(ws->dev, n_src, n_t, 0, sizeof(SrcDL64),
                                   mixed ? sizeof(SrcDL32) : 0, P.n_chunks);
    if (flags & STOKES_CHECK_INPUTS) {
        hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, S.flag);
        Check c{S.flag, st};
        c.finite(src_xyz, 3 * n_src);
        c.finite(src_normal, 3 * n_src);
        c.finite(src_weight, n_src);
        c.finite(src_q, 3 * n_src);
        if (!same) c.finite(trg_xyz, 3 * n_t);
        STOKES_HIP(hipGetLastError());
        int f = 0;
        if ((rc = read_flag(ws, S.flag, st, &f))) return rc;
        if (f & 1) return fail(STOKES_E_NONFINITE, "stokes_dl_eval: non-finite input");
    }
    unsigned long long* counters = diag ? S.counters : nullptr;
    if (counters) hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, counters, 4);
    const double* tx = same ? src_xyz : trg_xyz;
    const int64_t ts = same ? n_src : n_t;
    // tiles, packs and exclusion ranges in one launch (tiles only when there are sources)
    PrepArgs q{};
    q.n_s = n_src;
    q.sx = src_xyz;
    q.n_tiles = P.n_chunks > 0 ? P.n_tiles : 0;
    q.tile_blocks = P.n_chunks > 0 ? tile_prep_blocks(P.n_tiles) : 0;
    q.near_r = mixed ? nr : 0.0;
    q.near_fac = 0.0;
    q.band = mixed ? -1.0 : 0.0;
    q.nrm = src_normal;
    q.tiles = S.tiles;
    q.f = src_q;
    q.w = src_weight;
    q.sid = src_sid;
    q.s64 = S.s64;
    q.s32 = mixed ? S.s32 : nullptr;
    q.n_t = n_t;
    q.tself = trg_self;
    q.identity = same ? 1 : 0;
    q.excl = S.excl;
    q.counters = counters;
    hipLaunchKernelGGL(prep_kernel<true>, dim3(prep_grid(q)), dim3(TILE_PREP_BLOCK), 0, st, q);
    if (P.n_chunks > 0) {
        SumArgs a{};
        a.tx = tx;
        a.t_stride = ts;
        a.n_t = n_t;
        a.excl = S.excl;
        a.tiles = S.tiles;
        a.n_tiles = P.n_tiles;
        a.tiles_per_chunk = P.tiles_per_chunk;
        a.n_tblocks = P.n_tblocks;
        a.s64 = S.s64;
        a.s32 = S.s32;
        a.near_t_uniform = (float)(nr * nr);
        a.q = src_q;
        a.n_s = n_src;
        a.partial = S.partial;
        a.counters = counters;
        const unsigned grid = (unsigned)((int64_t)P.n_tblocks * P.n_chunks);
        if ((rc = check_grid(P, grid, n_t))) return rc;
        prof_begin(st);
        launch_dl_kernel(mixed, sub, src_sid != nullptr && sub, grid, a, st);
        prof_end(st);
    }
    hipLaunchKernelGGL(reduce_kernel, dim3(red_blocks(n_t)), dim3(RED_T * RED_S), 0, st, n_t, P.n_chunks,
                       S.partial, (flags & STOKES_ACCUMULATE) ? 1 : 0, u_out, n_t,
                       (const int2*)S.excl, sub ? src_q : (const double*)nullptr, n_src, -0.5,
                       mixed ? 1 : 0);
    STOKES_HIP(hipGetLastError());
    if (diag) return finish_diag(ws, counters, st, n_t, n_src, diag);
    return STOKES_OK;
}

extern "C" int stokes_dl_eval(int64_t n_src, const double* src_xyz, const double* src_normal,
                              const double* src_weight, const double* src_q, int64_t n_trg,
                              const double* trg_xyz, const int64_t* trg_self, double near_r,
                              uint32_t flags, double* u_out, void* stream, stokes_diag* diag) {
    return dl_run(n_src, src_xyz, src_normal, src_weight, src_q, nullptr, n_trg, trg_xyz, trg_self, near_r,
                  flags, u_out, stream, diag);
}

namespace stokes {

// Density of the double-layer packs: the only part of a plan's sources that changes
// between evaluations on a fixed geometry.
__global__ void dl_q_pack_kernel(int64_t n_s, const double* __restrict__ q, SrcDL64* s64, SrcDL32* s32) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_s) return;
    const double qx = q[j], qy = q[n_s + j], qz = q[2 * n_s + j];
    s64[j].qx = qx;
    s64[j].qy = qy;
    s64[j].qz = qz;
    if (s32) {
        s32[j].qx = (float)qx;
        s32[j].qy = (float)qy;
        s32[j].qz = (float)qz;
    }
}

DLPlan::~DLPlan() {
    if (mem_) (void)hipFree(mem_);
}

int DLPlan::init(int64_t n_src, const double* src_xyz, const double* src_normal, const double* src_weight,
                 const int32_t* src_sid, int64_t n_trg, const double* trg_xyz, const int64_t* trg_self,
                 double near_r, uint32_t flags, hipStream_t st) {
    if (mem_) return fail(STOKES_E_INVAL, "DLPlan::init: plan already made");
    const uint32_t known = STOKES_PREC_MIXED | STOKES_ONSURF_RAW;
    if (flags & ~known) return fail(STOKES_E_INVAL, "DLPlan::init: unknown flag bits");
    if (n_src < 1 || n_trg < 1 || !src_xyz || !src_normal || !src_weight || !trg_xyz)
        return fail(STOKES_E_INVAL, "DLPlan::init: empty or null geometry");
    if (n_src >= (int64_t)1 << 31 || n_trg >= (int64_t)1 << 31)
        return fail(STOKES_E_INVAL, "DLPlan::init: more than 2^31-1 sources or targets");
    if (src_sid && (flags & STOKES_ONSURF_RAW))
        return fail(STOKES_E_INVAL, "DLPlan::init: surface ids need the on-surface subtraction");
    mixed_ = flags & STOKES_PREC_MIXED;
    sub_ = !(flags & STOKES_ONSURF_RAW);
    multi_ = src_sid != nullptr;
    n_s_ = n_src;
    n_t_ = n_trg;
    txyz_ = trg_xyz;
    const double nr = near_r > 0.0 ? near_r : 0.02;
    near2_ = (float)(nr * nr);
    P_ = make_partition(n_t_, n_s_, mixed_ ? R_DL32 : R_DL64, TARGET_BLOCKS, 1, MIN_TILES_PER_CHUNK_DL);
    const SumLayout L = sum_layout(n_s_, n_t_, 0, sizeof(Tile), sizeof(SrcDL64), mixed_ ? sizeof(SrcDL32) : 0,
                                   P_.n_chunks);
    STOKES_HIP(hipMalloc(&mem_, L.bytes));
    char* b = static_cast<char*>(mem_);
    tiles_ = reinterpret_cast<Tile*>(b + L.tiles);
    s64_ = reinterpret_cast<SrcDL64*>(b + L.s64);
    s32_ = mixed_ ? reinterpret_cast<SrcDL32*>(b + L.s32) : nullptr;
    excl_ = reinterpret_cast<int2*>(b + L.excl);
    partial_ = reinterpret_cast<double*>(b + L.partial);
    // tiles, exclusion ranges, and positions, weighted normals and surface ids now; the
    // density per evaluation (the pack reads a density, so the normals stand in for it
    // until every evaluation overwrites them)
    PrepArgs q{};
    q.n_s = n_s_;
    q.sx = src_xyz;
    q.n_tiles = P_.n_tiles;
    q.tile_blocks = tile_prep_blocks(P_.n_tiles);
    q.near_r = mixed_ ? nr : 0.0;
    q.near_fac = 0.0;
    q.band = mixed_ ? -1.0 : 0.0;
    q.nrm = src_normal;
    q.tiles = tiles_;
    q.f = src_normal;
    q.w = src_weight;
    q.sid = src_sid;
    q.s64 = s64_;
    q.s32 = s32_;
    q.n_t = n_t_;
    q.tself = trg_self;
    q.identity = 0;
    q.excl = excl_;
    hipLaunchKernelGGL(prep_kernel<true>, dim3(prep_grid(q)), dim3(TILE_PREP_BLOCK), 0, st, q);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

int DLPlan::eval(const double* src_q, double* u_out, bool accumulate, hipStream_t st, bool in_capture) {
    if (!mem_) return fail(STOKES_E_INVAL, "DLPlan::eval: no plan");
    if (!src_q || !u_out) return fail(STOKES_E_INVAL, "DLPlan::eval: null pointer");
    hipLaunchKernelGGL(dl_q_pack_kernel, dim3(nblk(n_s_)), dim3(256), 0, st, n_s_, src_q, s64_, s32_);
    SumArgs a{};
    a.tx = txyz_;
    a.t_stride = n_t_;
    a.n_t = n_t_;
    a.excl = excl_;
    a.tiles = tiles_;
    a.n_tiles = P_.n_tiles;
    a.tiles_per_chunk = P_.tiles_per_chunk;
    a.n_tblocks = P_.n_tblocks;
    a.s64 = s64_;
    a.s32 = s32_;
    a.near_t_uniform = near2_;
    a.q = src_q;
    a.n_s = n_s_;
    a.partial = partial_;
    a.counters = nullptr;
    const unsigned grid = (unsigned)P_.grid();
    if (int rc = check_grid(P_, grid, n_t_)) return rc;
    if (!in_capture) prof_begin(st);
    launch_dl_kernel(mixed_, sub_, multi_, grid, a, st);
    if (!in_capture) prof_end(st);
    hipLaunchKernelGGL(reduce_kernel, dim3(red_blocks(n_t_)), dim3(RED_T * RED_S), 0, st, n_t_, P_.n_chunks,
                       (const double*)partial_, accumulate ? 1 : 0, u_out, n_t_, (const int2*)excl_,
                       sub_ ? src_q : (const double*)nullptr, n_s_, -0.5, mixed_ ? 1 : 0);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

}  // namespace stokes
