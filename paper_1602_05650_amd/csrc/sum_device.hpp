// Device code of the kernel sums, shared by the one-shot launches and the
// batched (serving) kernels.  See stokes_sums.hip for the execution scheme.
#pragma once

#include <climits>

#include "pair_math.hpp"
#include "stokes_internal.hpp"

// Unroll depth of the branch-free source loops (tuned on gfx950; overridable
// at compile time for experiments).
#ifndef STOKES_UNROLL_SL64
#define STOKES_UNROLL_SL64 4
#endif
#ifndef STOKES_UNROLL_SL32
#define STOKES_UNROLL_SL32 2
#endif
#ifndef STOKES_UNROLL_DL64
#define STOKES_UNROLL_DL64 2
#endif
#ifndef STOKES_UNROLL_DL32
#define STOKES_UNROLL_DL32 4
#endif

namespace stokes {

// Read-only view of device memory in the constant address space.  Used for
// buffers that no thread writes while the kernel runs (source packs, tiles,
// descriptor tables): the compiler then turns wave-uniform reads of them into
// scalar loads even when the kernel also stores to global memory.
// (The host compilation pass sees plain const pointers: these functions only
// run on the device.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using cptr = const __attribute__((address_space(4))) T*;
#else
template <class T>
using cptr = const T*;
#endif
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)p;
}

constexpr double PI_D = 3.14159265358979323846264338327950288;

// ---- small device helpers -------------------------------------------------

__device__ __forceinline__ bool in_range(int j, int lo, int hi) {
    return (unsigned)(j - lo) < (unsigned)(hi - lo);
}

// Squared distance of a tile-local point from the tile's capsule axis (FP32).
__device__ __forceinline__ float capsule_d2(const Tile& T, float x, float y, float z) {
    const float qx = x - T.ax, qy = y - T.ay, qz = z - T.az;
    float u = fmaf(qx, T.bx, fmaf(qy, T.by, qz * T.bz)) * T.inv_l2;
    u = fminf(fmaxf(u, 0.0f), 1.0f);
    const float dx = fmaf(-u, T.bx, qx), dy = fmaf(-u, T.by, qy), dz = fmaf(-u, T.bz, qz);
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

__device__ __forceinline__ void kahan_add(float& S, float& C, float v) {
    const float y = v - C;
    const float t = S + y;
    C = (t - S) - y;
    S = t;
}

// Single-layer pair, FP64: u += s/r + c s/r^3 + d (d.s) (1/r^3 - 3c/r^5).
template <bool DOUBLET>
__device__ __forceinline__ void sl_pair64(double dx, double dy, double dz, double ri,
                                          const SrcSL64& s, double& ux, double& uy, double& uz) {
    const double ri2 = ri * ri;
    const double ri3 = ri * ri2;
    const double ds = fma(dx, s.sx, fma(dy, s.sy, dz * s.sz));
    double A, E;
    if (DOUBLET) {
        const double ri5 = ri3 * ri2;
        A = fma(s.c, ri3, ri);
        E = fma(s.c3, ri5, ri3);
    } else {
        A = ri;
        E = ri3;
    }
    const double B = ds * E;
    ux = fma(A, s.sx, ux);
    uy = fma(A, s.sy, uy);
    uz = fma(A, s.sz, uz);
    ux = fma(B, dx, ux);
    uy = fma(B, dy, uy);
    uz = fma(B, dz, uz);
}

template <bool DOUBLET>
__device__ __forceinline__ void sl_pair32(float dx, float dy, float dz, float ri,
                                          const SrcSL32& s, float& ux, float& uy, float& uz) {
    const float ri2 = ri * ri;
    const float ri3 = ri * ri2;
    const float ds = fmaf(dx, s.sx, fmaf(dy, s.sy, dz * s.sz));
    float A, E;
    if (DOUBLET) {
        const float ri5 = ri3 * ri2;
        A = fmaf(s.c, ri3, ri);
        E = fmaf(s.c3, ri5, ri3);
    } else {
        A = ri;
        E = ri3;
    }
    const float B = ds * E;
    ux = fmaf(A, s.sx, ux);
    uy = fmaf(A, s.sy, uy);
    uz = fmaf(A, s.sz, uz);
    ux = fmaf(B, dx, ux);
    uy = fmaf(B, dy, uy);
    uz = fmaf(B, dz, uz);
}

// Double-layer pair: u += (d.qt)(d.n') d / r^5 with n' = (3/(4 pi)) w n.
template <bool SUB>
__device__ __forceinline__ void dl_pair64(double dx, double dy, double dz, double ri,
                                          const SrcDL64& s, double q0x, double q0y, double q0z,
                                          double& ux, double& uy, double& uz) {
    const double qx = SUB ? s.qx - q0x : s.qx;
    const double qy = SUB ? s.qy - q0y : s.qy;
    const double qz = SUB ? s.qz - q0z : s.qz;
    const double dq = fma(dx, qx, fma(dy, qy, dz * qz));
    const double dn = fma(dx, s.nx, fma(dy, s.ny, dz * s.nz));
    const double ri2 = ri * ri;
    const double ri5 = ri2 * ri2 * ri;
    const double e = dq * dn * ri5;
    ux = fma(e, dx, ux);
    uy = fma(e, dy, uy);
    uz = fma(e, dz, uz);
}

// FP32 pair with d.n' given (dl_pair32 forms it from the FP32 operands).
template <bool SUB>
__device__ __forceinline__ void dl_pair32_dn(float dx, float dy, float dz, float dn, float r2, float ri,
                                             const SrcDL32& s, float q0x, float q0y, float q0z,
                                             float& ux, float& uy, float& uz) {
    const float qx = SUB ? s.qx - q0x : s.qx;
    const float qy = SUB ? s.qy - q0y : s.qy;
    const float qz = SUB ? s.qz - q0z : s.qz;
    const float dq = fmaf(dx, qx, fmaf(dy, qy, dz * qz));
    const float e = dq * dn * rinv5_f32(r2, ri);
    ux = fmaf(e, dx, ux);
    uy = fmaf(e, dy, uy);
    uz = fmaf(e, dz, uz);
}

template <bool SUB>
__device__ __forceinline__ void dl_pair32(float dx, float dy, float dz, float r2, float ri, const SrcDL32& s,
                                          float q0x, float q0y, float q0z, float& ux, float& uy,
                                          float& uz) {
    const float dn = fmaf(dx, s.nx, fmaf(dy, s.ny, dz * s.nz));
    dl_pair32_dn<SUB>(dx, dy, dz, dn, r2, ri, s, q0x, q0y, q0z, ux, uy, uz);
}

__device__ __forceinline__ void wave_count(unsigned long long* ctr, unsigned long long v) {
    // one atomic per wave and counter (integer: order-independent)
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(ctr, v);
}

// Union of the lanes' non-empty exclusion ranges [lo, hi) of a wave, wave-uniform (an
// empty union has x > y).  A tile that misses it needs no exclusion test; one that
// meets it takes the checked path, which tests every pair.  Call with the whole wave.
template <int R>
__device__ __forceinline__ int2 wave_excl_union(const int (&lo)[R], const int (&hi)[R]) {
    int a = INT_MAX, b = INT_MIN;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (hi[r] > lo[r]) {
            a = min(a, lo[r]);
            b = max(b, hi[r]);
        }
    for (int off = 32; off > 0; off >>= 1) {
        a = min(a, __shfl_xor(a, off, 64));
        b = max(b, __shfl_xor(b, off, 64));
    }
    return make_int2(__builtin_amdgcn_readfirstlane(a), __builtin_amdgcn_readfirstlane(b));
}

// ---- kernel arguments -------------------------------------------------------
struct SumArgs {
    const double* tx;        // target planes: tx[c * t_stride + i]
    int64_t t_stride;
    int64_t n_t;
    const int2* excl;        // per-target excluded source range [lo, hi), or null
    const Tile* tiles;
    int32_t n_tiles;
    int32_t tiles_per_chunk;
    int32_t n_tblocks;
    const void* s64;         // SrcSL64 / SrcDL64
    const void* s32;         // SrcSL32 / SrcDL32 (mixed)
    const float* near_t;     // SL mixed: per-source FP32 near threshold on |d|^2
    float near_t_uniform;    // DL mixed: threshold on |d|^2
    const double* q;         // DL: density planes (for q_self), stride n_s
    int64_t n_s;
    double* partial;         // [n_chunks][3][n_t]
    unsigned long long* counters;  // null or {near, coincident, excluded}
};

// ---- single layer, FP64 -------------------------------------------------------
template <int R, bool DOUBLET>
__device__ __forceinline__ void sl_fp64_wave(const SumArgs& a, int tb, int chunk) {
    const int lane = threadIdx.x & 63;
    const int64_t wbase = ((int64_t)tb * 4 + (threadIdx.x >> 6)) * (64 * R);
    if (wbase >= a.n_t) return;

    double X[R], Y[R], Z[R], ux[R], uy[R], uz[R];
    int lo[R], hi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t i = wbase + lane + 64 * r;
        if (i >= a.n_t) i = a.n_t - 1;
        X[r] = a.tx[i];
        Y[r] = a.tx[a.t_stride + i];
        Z[r] = a.tx[2 * a.t_stride + i];
        const int2 e = a.excl ? a.excl[i] : make_int2(0, 0);
        lo[r] = e.x;
        hi[r] = e.y;
        ux[r] = uy[r] = uz[r] = 0.0;
    }
    uint32_t ncoin = 0;
    const cptr<SrcSL64> src = as_const(static_cast<const SrcSL64*>(a.s64));
    const int2 xu = wave_excl_union<R>(lo, hi);
    const int t0 = chunk * a.tiles_per_chunk;
    const int t1 = min(t0 + a.tiles_per_chunk, a.n_tiles);
    for (int t = t0; t < t1; ++t) {
        const Tile T = as_const(a.tiles)[t];
        bool near_s = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double dx = X[r] - T.ox, dy = Y[r] - T.oy, dz = Z[r] - T.oz;
            near_s |= fma(dx, dx, fma(dy, dy, dz * dz)) <= T.reach2;
        }
        // wave-uniform: the union of the lanes' exclusion ranges overlaps the tile
        bool checked = (xu.x < T.j1) & (xu.y > T.j0);
        if (__ballot(near_s) != 0) {   // refine the sphere test with the capsule
            bool near_c = false;
#pragma unroll
            for (int r = 0; r < R; ++r)
                near_c |= capsule_d2(T, (float)(X[r] - T.ox), (float)(Y[r] - T.oy),
                                     (float)(Z[r] - T.oz)) <= T.cap2_d;
            checked |= __ballot(near_s & near_c) != 0;
        }
        if (!checked) {
#pragma unroll STOKES_UNROLL_SL64
            for (int j = T.j0; j < T.j1; ++j) {
                const SrcSL64 s = src[j];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double dx = X[r] - s.x, dy = Y[r] - s.y, dz = Z[r] - s.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    sl_pair64<DOUBLET>(dx, dy, dz, rsqrt64(r2), s, ux[r], uy[r], uz[r]);
                }
            }
        } else {
            for (int j = T.j0; j < T.j1; ++j) {
                const SrcSL64 s = src[j];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double dx = X[r] - s.x, dy = Y[r] - s.y, dz = Z[r] - s.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    const bool ex = in_range(j, lo[r], hi[r]);
                    const bool zero = (r2 == 0.0);
                    ncoin += (!ex && zero && (wbase + lane + 64 * r < a.n_t)) ? 1 : 0;
                    const double ri = (ex || zero) ? 0.0 : rsqrt64(zero ? 1.0 : r2);
                    sl_pair64<DOUBLET>(dx, dy, dz, ri, s, ux[r], uy[r], uz[r]);
                }
            }
        }
    }
    double* out = a.partial + (int64_t)chunk * 3 * a.n_t;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = wbase + lane + 64 * r;
        if (i < a.n_t) {
            out[i] = ux[r];
            out[a.n_t + i] = uy[r];
            out[2 * a.n_t + i] = uz[r];
        }
    }
    if (a.counters) wave_count(a.counters + 1, ncoin);
}

// ---- single layer, mixed FP32 / FP64 -------------------------------------------
template <int R, bool DOUBLET>
__device__ __forceinline__ void sl_mixed_wave(const SumArgs& a, int tb, int chunk) {
    const int lane = threadIdx.x & 63;
    const int64_t wbase = ((int64_t)tb * 4 + (threadIdx.x >> 6)) * (64 * R);
    const bool wave_active = wbase < a.n_t;   // else only the barrier loop below
    // source tile staged in LDS: every operand of the pair arithmetic is a VGPR
    // (gfx950 issues FP32 VALU ops with an SGPR operand at a lower rate)
    __shared__ float4 lds[2 * TILE];
    // FP64 near-pair sums and counts of each thread: touched only on the rare checked
    // tiles, so they live in the thread's own LDS slots, not in loop-carried registers
    __shared__ double near_sum[3 * R][BLOCK];
    __shared__ uint32_t near_cnt[2][BLOCK];
    const int tid = threadIdx.x;

    double X[R], Y[R], Z[R];
    float Sx[R], Sy[R], Sz[R], Cx[R], Cy[R], Cz[R];
    int lo[R], hi[R];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t i = wbase + lane + 64 * r;
        valid[r] = i < a.n_t;
        if (!valid[r]) i = a.n_t - 1;
        X[r] = a.tx[i];
        Y[r] = a.tx[a.t_stride + i];
        Z[r] = a.tx[2 * a.t_stride + i];
        const int2 e = a.excl ? a.excl[i] : make_int2(0, 0);
        lo[r] = e.x;
        hi[r] = e.y;
        near_sum[3 * r][tid] = near_sum[3 * r + 1][tid] = near_sum[3 * r + 2][tid] = 0.0;
        Sx[r] = Sy[r] = Sz[r] = Cx[r] = Cy[r] = Cz[r] = 0.0f;
    }
    near_cnt[0][tid] = near_cnt[1][tid] = 0u;   // at most the thread's targets x the chunk's sources
    const cptr<float4> src4 = as_const(static_cast<const float4*>(a.s32));
    const SrcSL64* __restrict__ src64 = static_cast<const SrcSL64*>(a.s64);
    const int2 xu = wave_excl_union<R>(lo, hi);
    const int t0 = chunk * a.tiles_per_chunk;
    const int t1 = min(t0 + a.tiles_per_chunk, a.n_tiles);
    if (!wave_active) {   // a wave past the targets still stages tiles and meets the barriers
        for (int t = t0; t < t1; ++t) {
            const Tile T = as_const(a.tiles)[t];
            const int nsrc = T.j1 - T.j0;
            if ((int)threadIdx.x < 2 * nsrc) lds[threadIdx.x] = src4[2 * (int64_t)T.j0 + threadIdx.x];
            __syncthreads();
            __syncthreads();
        }
        return;
    }
    // FP32 partial of two consecutive tiles, added to the Kahan pair after every second
    // tile and after the chunk's last
    float px[R], py[R], pz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) px[r] = py[r] = pz[r] = 0.0f;
    for (int t = t0; t < t1; ++t) {
        const Tile T = as_const(a.tiles)[t];
        const int nsrc = T.j1 - T.j0;
        if ((int)threadIdx.x < 2 * nsrc) lds[threadIdx.x] = src4[2 * (int64_t)T.j0 + threadIdx.x];
        __syncthreads();
        float xs[R], ys[R], zs[R];
        bool near_s = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            xs[r] = (float)(X[r] - T.ox);
            ys[r] = (float)(Y[r] - T.oy);
            zs[r] = (float)(Z[r] - T.oz);
            near_s |= fmaf(xs[r], xs[r], fmaf(ys[r], ys[r], zs[r] * zs[r])) <= T.reach2_f;
        }
        // wave-uniform: the union of the lanes' exclusion ranges overlaps the tile
        bool checked = (xu.x < T.j1) & (xu.y > T.j0);
        if (__ballot(near_s) != 0) {   // refine the sphere test with the capsule
            bool near_c = false;
#pragma unroll
            for (int r = 0; r < R; ++r) near_c |= capsule_d2(T, xs[r], ys[r], zs[r]) <= T.cap2_f;
            checked |= __ballot(near_s & near_c) != 0;
        }
        if (!checked) {
            auto far = [&](int k) {
                const float4 p0 = lds[2 * k], p1 = lds[2 * k + 1];
                const SrcSL32 s = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float dx = xs[r] - s.x, dy = ys[r] - s.y, dz = zs[r] - s.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    sl_pair32<DOUBLET>(dx, dy, dz, __builtin_amdgcn_rsqf(r2), s, px[r], py[r], pz[r]);
                }
            };
            if (nsrc == TILE) {   // a full tile: LDS addresses are immediate offsets
#pragma unroll
                for (int k = 0; k < TILE; ++k) far(k);
            } else {
#pragma unroll STOKES_UNROLL_SL32
                for (int k = 0; k < nsrc; ++k) far(k);
            }
        } else {
            uint32_t m[R];
#pragma unroll
            for (int r = 0; r < R; ++r) m[r] = 0u;
            for (int k = 0; k < nsrc; ++k) {
                const int j = T.j0 + k;
                const float4 p0 = lds[2 * k], p1 = lds[2 * k + 1];
                const SrcSL32 s = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
                const float tj = as_const(a.near_t)[j];
                const uint32_t bit = 1u << k;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float dx = xs[r] - s.x, dy = ys[r] - s.y, dz = zs[r] - s.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const bool bad = (r2 < tj) | in_range(j, lo[r], hi[r]);
                    m[r] |= bad ? bit : 0u;
                    const float ri = bad ? 0.0f : __builtin_amdgcn_rsqf(r2);
                    sl_pair32<DOUBLET>(dx, dy, dz, ri, s, px[r], py[r], pz[r]);
                }
            }
            // FP64 recomputation of the masked (near) pairs from the FP64 inputs
            uint32_t nnear = 0, ncoin = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double ax = 0.0, ay = 0.0, az = 0.0;
                uint32_t mm = m[r];
                while (mm) {
                    const int k = __builtin_ctz(mm);
                    mm &= mm - 1;
                    const int j = T.j0 + k;
                    if (in_range(j, lo[r], hi[r])) continue;
                    const SrcSL64 s = src64[j];
                    const double dx = X[r] - s.x, dy = Y[r] - s.y, dz = Z[r] - s.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    if (r2 == 0.0) {
                        ncoin += valid[r] ? 1 : 0;
                        continue;
                    }
                    nnear += valid[r] ? 1 : 0;
                    sl_pair64<DOUBLET>(dx, dy, dz, rsqrt64(r2), s, ax, ay, az);
                }
                near_sum[3 * r][tid] += ax;
                near_sum[3 * r + 1][tid] += ay;
                near_sum[3 * r + 2][tid] += az;
            }
            near_cnt[0][tid] += nnear;
            near_cnt[1][tid] += ncoin;
        }
        if (((t - t0) & 1) || t == t1 - 1) {   // wave-uniform
#pragma unroll
            for (int r = 0; r < R; ++r) {
                kahan_add(Sx[r], Cx[r], px[r]);
                kahan_add(Sy[r], Cy[r], py[r]);
                kahan_add(Sz[r], Cz[r], pz[r]);
                px[r] = py[r] = pz[r] = 0.0f;
            }
        }
        __syncthreads();
    }
    double* out = a.partial + (int64_t)chunk * 3 * a.n_t;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = wbase + lane + 64 * r;
        if (valid[r]) {
            out[i] = ((double)Sx[r] - (double)Cx[r]) + near_sum[3 * r][tid];
            out[a.n_t + i] = ((double)Sy[r] - (double)Cy[r]) + near_sum[3 * r + 1][tid];
            out[2 * a.n_t + i] = ((double)Sz[r] - (double)Cz[r]) + near_sum[3 * r + 2][tid];
        }
    }
    if (a.counters) {
        wave_count(a.counters + 0, near_cnt[0][tid]);
        wave_count(a.counters + 1, near_cnt[1][tid]);
    }
}

// ---- double layer, FP64 -----------------------------------------------------
// MULTI: the sources are several surfaces, their ids in SrcDL64::pad0; a target's own
// density (SUB) is subtracted only from the sources of its own surface, the surface
// of its self source (a target without one takes every source raw).
template <int R, bool SUB, bool MULTI = false>
__device__ __forceinline__ void dl_fp64_wave(const SumArgs& a, int tb, int chunk) {
    const int lane = threadIdx.x & 63;
    const int64_t wbase = ((int64_t)tb * 4 + (threadIdx.x >> 6)) * (64 * R);
    if (wbase >= a.n_t) return;

    double X[R], Y[R], Z[R], ux[R], uy[R], uz[R], qx[R], qy[R], qz[R], tsid[R];
    int lo[R], hi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t i = wbase + lane + 64 * r;
        if (i >= a.n_t) i = a.n_t - 1;
        X[r] = a.tx[i];
        Y[r] = a.tx[a.t_stride + i];
        Z[r] = a.tx[2 * a.t_stride + i];
        const int2 e = a.excl ? a.excl[i] : make_int2(0, 0);
        lo[r] = e.x;
        hi[r] = e.y;
        qx[r] = qy[r] = qz[r] = 0.0;
        tsid[r] = -1.0;
        if (SUB && e.y > e.x) {
            qx[r] = a.q[e.x];
            qy[r] = a.q[a.n_s + e.x];
            qz[r] = a.q[2 * a.n_s + e.x];
            if (MULTI) tsid[r] = static_cast<const SrcDL64*>(a.s64)[e.x].pad0;
        }
        ux[r] = uy[r] = uz[r] = 0.0;
    }
    uint32_t ncoin = 0;
    const cptr<SrcDL64> src = as_const(static_cast<const SrcDL64*>(a.s64));
    const int2 xu = wave_excl_union<R>(lo, hi);
    const int t0 = chunk * a.tiles_per_chunk;
    const int t1 = min(t0 + a.tiles_per_chunk, a.n_tiles);
    for (int t = t0; t < t1; ++t) {
        const Tile T = as_const(a.tiles)[t];
        bool near_s = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double dx = X[r] - T.ox, dy = Y[r] - T.oy, dz = Z[r] - T.oz;
            near_s |= fma(dx, dx, fma(dy, dy, dz * dz)) <= T.reach2;
        }
        // wave-uniform: the union of the lanes' exclusion ranges overlaps the tile
        bool checked = (xu.x < T.j1) & (xu.y > T.j0);
        if (__ballot(near_s) != 0) {   // refine the sphere test with the capsule
            bool near_c = false;
#pragma unroll
            for (int r = 0; r < R; ++r)
                near_c |= capsule_d2(T, (float)(X[r] - T.ox), (float)(Y[r] - T.oy),
                                     (float)(Z[r] - T.oz)) <= T.cap2_d;
            checked |= __ballot(near_s & near_c) != 0;
        }
        if (!checked) {
#pragma unroll STOKES_UNROLL_DL64
            for (int j = T.j0; j < T.j1; ++j) {
                const SrcDL64 s = src[j];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double dx = X[r] - s.x, dy = Y[r] - s.y, dz = Z[r] - s.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    const bool own = !MULTI || s.pad0 == tsid[r];
                    dl_pair64<SUB>(dx, dy, dz, rsqrt64(r2), s, own ? qx[r] : 0.0, own ? qy[r] : 0.0,
                                   own ? qz[r] : 0.0, ux[r], uy[r], uz[r]);
                }
            }
        } else {
            for (int j = T.j0; j < T.j1; ++j) {
                const SrcDL64 s = src[j];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double dx = X[r] - s.x, dy = Y[r] - s.y, dz = Z[r] - s.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    const bool ex = in_range(j, lo[r], hi[r]);
                    const bool zero = (r2 == 0.0);
                    ncoin += (!ex && zero && (wbase + lane + 64 * r < a.n_t)) ? 1 : 0;
                    const double ri = (ex || zero) ? 0.0 : rsqrt64(zero ? 1.0 : r2);
                    const bool own = !MULTI || s.pad0 == tsid[r];
                    dl_pair64<SUB>(dx, dy, dz, ri, s, own ? qx[r] : 0.0, own ? qy[r] : 0.0, own ? qz[r] : 0.0,
                                   ux[r], uy[r], uz[r]);
                }
            }
        }
    }
    double* out = a.partial + (int64_t)chunk * 3 * a.n_t;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = wbase + lane + 64 * r;
        if (i < a.n_t) {
            out[i] = ux[r];
            out[a.n_t + i] = uy[r];
            out[2 * a.n_t + i] = uz[r];
        }
    }
    if (a.counters) wave_count(a.counters + 1, ncoin);
}

// ---- double layer, mixed FP32 / FP64 -------------------------------------------
// MULTI as for dl_fp64_wave (the FP32 pack carries the surface id in pad0 too).
template <int R, bool SUB, bool MULTI = false>
__device__ __forceinline__ void dl_mixed_wave(const SumArgs& a, int tb, int chunk) {
    const int lane = threadIdx.x & 63;
    const int64_t wbase = ((int64_t)tb * 4 + (threadIdx.x >> 6)) * (64 * R);
    const bool wave_active = wbase < a.n_t;   // else only the barrier loop below
    // source tile staged in LDS: every operand of the pair arithmetic is a VGPR
    // (gfx950 issues FP32 VALU ops with an SGPR operand at a lower rate)
    __shared__ float4 lds[3 * TILE];
    // the tile's FP64 positions and weighted normals (x, y | z, - | n'x, n'y | n'z, -) for
    // the loops that form d and d.n' in FP64; staged with the FP32 pack every tile
    __shared__ double2 lds64[4 * TILE];
    // FP64 near-pair sums and counts of each thread: touched only on the rare checked
    // tiles, so they live in the thread's own LDS slots, not in loop-carried registers
    __shared__ double near_sum[3 * R][BLOCK];
    __shared__ uint32_t near_cnt[2][BLOCK];
    const int tid = threadIdx.x;

    double X[R], Y[R], Z[R], qx[R], qy[R], qz[R], tsid[R];
    float fqx[R], fqy[R], fqz[R];
    float Sx[R], Sy[R], Sz[R], Cx[R], Cy[R], Cz[R];
    int lo[R], hi[R];
    bool valid[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t i = wbase + lane + 64 * r;
        valid[r] = i < a.n_t;
        if (!valid[r]) i = a.n_t - 1;
        X[r] = a.tx[i];
        Y[r] = a.tx[a.t_stride + i];
        Z[r] = a.tx[2 * a.t_stride + i];
        const int2 e = a.excl ? a.excl[i] : make_int2(0, 0);
        lo[r] = e.x;
        hi[r] = e.y;
        qx[r] = qy[r] = qz[r] = 0.0;
        tsid[r] = -1.0;
        if (SUB && e.y > e.x) {
            qx[r] = a.q[e.x];
            qy[r] = a.q[a.n_s + e.x];
            qz[r] = a.q[2 * a.n_s + e.x];
            if (MULTI) tsid[r] = static_cast<const SrcDL64*>(a.s64)[e.x].pad0;
        }
        // The subtracted self density is rounded to FP32 once, and that value is used by
        // the FP32 pairs, the FP64 near pairs and the jump term (reduce_kernel) alike:
        // the constant part of q then cancels against the jump up to the discrete
        // identity's defect, instead of leaving half the rounding of q_self behind.
        fqx[r] = (float)qx[r];
        fqy[r] = (float)qy[r];
        fqz[r] = (float)qz[r];
        qx[r] = (double)fqx[r];
        qy[r] = (double)fqy[r];
        qz[r] = (double)fqz[r];
        near_sum[3 * r][tid] = near_sum[3 * r + 1][tid] = near_sum[3 * r + 2][tid] = 0.0;
        Sx[r] = Sy[r] = Sz[r] = Cx[r] = Cy[r] = Cz[r] = 0.0f;
    }
    near_cnt[0][tid] = near_cnt[1][tid] = 0u;   // at most the thread's targets x the chunk's sources
    const cptr<float4> src4 = as_const(static_cast<const float4*>(a.s32));
    const SrcDL64* __restrict__ src64 = static_cast<const SrcDL64*>(a.s64);
    // double2 words 0, 1, 3, 4 of a 6-word SrcDL64: (x, y), (z, qx), (nx, ny), (nz, pad0)
    const cptr<double2> src2 = as_const(static_cast<const double2*>(a.s64));
    auto stage = [&](const Tile& T, int nsrc) {
        const int th = threadIdx.x;
        if (th < 3 * nsrc) lds[th] = src4[3 * (int64_t)T.j0 + th];
        const int u = th - 128;
        if (u >= 0 && u < 4 * nsrc) {
            const int k = u >> 2, w = u & 3;
            lds64[u] = src2[6 * ((int64_t)T.j0 + k) + (w < 2 ? w : w + 1)];
        }
    };
    const float tn = a.near_t_uniform;
    const int2 xu = wave_excl_union<R>(lo, hi);
    const int t0 = chunk * a.tiles_per_chunk;
    const int t1 = min(t0 + a.tiles_per_chunk, a.n_tiles);
    if (!wave_active) {   // a wave past the targets still stages tiles and meets the barriers
        for (int t = t0; t < t1; ++t) {
            const Tile T = as_const(a.tiles)[t];
            stage(T, T.j1 - T.j0);
            __syncthreads();
            __syncthreads();
        }
        return;
    }
    for (int t = t0; t < t1; ++t) {
        const Tile T = as_const(a.tiles)[t];
        const int nsrc = T.j1 - T.j0;
        stage(T, nsrc);
        __syncthreads();
        float xs[R], ys[R], zs[R], px[R], py[R], pz[R];
        bool near_s = false, band_s = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            xs[r] = (float)(X[r] - T.ox);
            ys[r] = (float)(Y[r] - T.oy);
            zs[r] = (float)(Z[r] - T.oz);
            const float d2 = fmaf(xs[r], xs[r], fmaf(ys[r], ys[r], zs[r] * zs[r]));
            near_s |= d2 <= T.reach2_f;
            band_s |= d2 <= T.band2_f;   // in the tile's tangent band
            px[r] = py[r] = pz[r] = 0.0f;
        }
        // wave-uniform: the union of the lanes' exclusion ranges overlaps the tile
        bool checked = (xu.x < T.j1) & (xu.y > T.j0);
        const bool band = __ballot(band_s) != 0;
        if (!checked && __ballot(near_s) != 0) {   // refine the sphere test with the capsule
            bool near_c = false;
#pragma unroll
            for (int r = 0; r < R; ++r) near_c |= capsule_d2(T, xs[r], ys[r], zs[r]) <= T.cap2_f;
            checked |= __ballot(near_s & near_c) != 0;
        }
        // FP64 d and d.n' (rounded once) for a pair of the tile, from the staged FP64 data.
        // Used in the tangent band, where d is nearly tangent to the surface and
        // d.n' ~ |d|^2 / (2 R_curv): from tile-local FP32 coordinates it would lose
        // ~ eps32 2 R_curv / |d| of itself, the largest rounding error of the mixed sum.
        auto d64 = [&](int k, int r, float& dx, float& dy, float& dz, float& dn) {
            const double2 a0 = lds64[4 * k], a1 = lds64[4 * k + 1], a2 = lds64[4 * k + 2], a3 = lds64[4 * k + 3];
            const double Dx = X[r] - a0.x, Dy = Y[r] - a0.y, Dz = Z[r] - a1.x;
            dx = (float)Dx;
            dy = (float)Dy;
            dz = (float)Dz;
            dn = (float)fma(Dx, a2.x, fma(Dy, a2.y, Dz * a3.x));
        };
        if (!checked && band) {   // no near or excluded pair: the band loop, without masks
            auto bpair = [&](int k) {
                const float4 p0 = lds[3 * k], p1 = lds[3 * k + 1], p2 = lds[3 * k + 2];
                const SrcDL32 s = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x, MULTI ? p2.y : 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float dx, dy, dz, dn;
                    d64(k, r, dx, dy, dz, dn);
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const bool own = !MULTI || s.pad0 == (float)tsid[r];
                    dl_pair32_dn<SUB>(dx, dy, dz, dn, r2, __builtin_amdgcn_rsqf(r2), s, own ? fqx[r] : 0.f,
                                      own ? fqy[r] : 0.f, own ? fqz[r] : 0.f, px[r], py[r], pz[r]);
                }
            };
#pragma unroll 2
            for (int k = 0; k < nsrc; ++k) bpair(k);
        } else if (!checked) {
            auto far = [&](int k) {
                const float4 p0 = lds[3 * k], p1 = lds[3 * k + 1], p2 = lds[3 * k + 2];
                const SrcDL32 s = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x, MULTI ? p2.y : 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float dx = xs[r] - s.x, dy = ys[r] - s.y, dz = zs[r] - s.z;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const bool own = !MULTI || s.pad0 == (float)tsid[r];
                    dl_pair32<SUB>(dx, dy, dz, r2, __builtin_amdgcn_rsqf(r2), s, own ? fqx[r] : 0.f, own ? fqy[r] : 0.f,
                                   own ? fqz[r] : 0.f,
                                   px[r], py[r], pz[r]);
                }
            };
            if (nsrc == TILE) {   // a full tile: LDS addresses are immediate offsets
#pragma unroll
                for (int k = 0; k < TILE; ++k) far(k);
            } else {
#pragma unroll STOKES_UNROLL_DL32
                for (int k = 0; k < nsrc; ++k) far(k);
            }
        } else {
            // checked loop: d and d.n' in FP64 as in the band loop; near and excluded pairs masked
            uint32_t m[R];
#pragma unroll
            for (int r = 0; r < R; ++r) m[r] = 0u;
            for (int k = 0; k < nsrc; ++k) {
                const int j = T.j0 + k;
                const float4 p0 = lds[3 * k], p1 = lds[3 * k + 1], p2 = lds[3 * k + 2];
                const SrcDL32 s = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x, MULTI ? p2.y : 0.f, 0.f, 0.f};
                const uint32_t bit = 1u << k;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    float dx, dy, dz, dn;
                    d64(k, r, dx, dy, dz, dn);
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const bool bad = (r2 < tn) | in_range(j, lo[r], hi[r]);
                    m[r] |= bad ? bit : 0u;
                    const float ri = bad ? 0.0f : __builtin_amdgcn_rsqf(r2);
                    const bool own = !MULTI || s.pad0 == (float)tsid[r];
                    dl_pair32_dn<SUB>(dx, dy, dz, dn, r2, ri, s, own ? fqx[r] : 0.f, own ? fqy[r] : 0.f,
                                      own ? fqz[r] : 0.f, px[r], py[r], pz[r]);
                }
            }
            uint32_t nnear = 0, ncoin = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double ax = 0.0, ay = 0.0, az = 0.0;
                uint32_t mm = m[r];
                while (mm) {
                    const int k = __builtin_ctz(mm);
                    mm &= mm - 1;
                    const int j = T.j0 + k;
                    if (in_range(j, lo[r], hi[r])) continue;
                    const SrcDL64 s = src64[j];
                    const double dx = X[r] - s.x, dy = Y[r] - s.y, dz = Z[r] - s.z;
                    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
                    if (r2 == 0.0) {
                        ncoin += valid[r] ? 1 : 0;
                        continue;
                    }
                    nnear += valid[r] ? 1 : 0;
                    const bool own = !MULTI || s.pad0 == tsid[r];
                    dl_pair64<SUB>(dx, dy, dz, rsqrt64(r2), s, own ? qx[r] : 0.0, own ? qy[r] : 0.0,
                                   own ? qz[r] : 0.0, ax, ay, az);
                }
                near_sum[3 * r][tid] += ax;
                near_sum[3 * r + 1][tid] += ay;
                near_sum[3 * r + 2][tid] += az;
            }
            near_cnt[0][tid] += nnear;
            near_cnt[1][tid] += ncoin;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            kahan_add(Sx[r], Cx[r], px[r]);
            kahan_add(Sy[r], Cy[r], py[r]);
            kahan_add(Sz[r], Cz[r], pz[r]);
        }
        __syncthreads();
    }
    double* out = a.partial + (int64_t)chunk * 3 * a.n_t;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = wbase + lane + 64 * r;
        if (valid[r]) {
            out[i] = ((double)Sx[r] - (double)Cx[r]) + near_sum[3 * r][tid];
            out[a.n_t + i] = ((double)Sy[r] - (double)Cy[r]) + near_sum[3 * r + 1][tid];
            out[2 * a.n_t + i] = ((double)Sz[r] - (double)Cz[r]) + near_sum[3 * r + 2][tid];
        }
    }
    if (a.counters) {
        wave_count(a.counters + 0, near_cnt[0][tid]);
        wave_count(a.counters + 1, near_cnt[1][tid]);
    }
}


// ---- preparation (per tile / per source) ----
__device__ __forceinline__ void tile_prep_one(int t, int64_t n_s, const double* __restrict__ sx,
                                              double near_r, double near_fac,
                                              const int32_t* __restrict__ sfib, int32_t n_fib,
                                              const double* __restrict__ flen, Tile* tiles,
                                              double band = 0.0) {
    const int j0 = t * TILE;
    const int j1 = (int)min((int64_t)j0 + TILE, n_s);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double nr = near_r;
    for (int j = j0; j < j1; ++j) {
        for (int c = 0; c < 3; ++c) {
            const double v = sx[c * n_s + j];
            lo[c] = fmin(lo[c], v);
            hi[c] = fmax(hi[c], v);
        }
        if (near_fac > 0.0) {
            double L = 1.0;
            if (flen) {
                int f = sfib ? sfib[j] : 0;
                if (f >= 0 && f < (sfib ? n_fib : 1)) L = flen[f];
            }
            nr = fmax(nr, near_fac * L);
        }
    }
    Tile T;
    T.ox = 0.5 * (lo[0] + hi[0]);
    T.oy = 0.5 * (lo[1] + hi[1]);
    T.oz = 0.5 * (lo[2] + hi[2]);
    double rad2 = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double dx = sx[j] - T.ox, dy = sx[n_s + j] - T.oy, dz = sx[2 * n_s + j] - T.oz;
        rad2 = fmax(rad2, dx * dx + dy * dy + dz * dz);
    }
    const double rad = sqrt(rad2);
    const double r64 = rad * (1.0 + 1e-9) + 1e-300;
    T.reach2 = r64 * r64;
    const double rm = (rad + nr) * (1.0 + 1e-5) + 1e-30;
    T.reach2_f = (float)(rm * rm) * (1.0f + 1e-6f);
    T.j0 = j0;
    T.j1 = j1;
    // capsule: axis from the first to the last source; radius = largest distance
    // of a source from that segment.  The FP32 test of a target against it
    // (in tile-local coordinates) gets a margin that covers its rounding.
    const double a[3] = {sx[j0] - T.ox, sx[n_s + j0] - T.oy, sx[2 * n_s + j0] - T.oz};
    const double b[3] = {sx[j1 - 1] - sx[j0], sx[n_s + j1 - 1] - sx[n_s + j0],
                         sx[2 * n_s + j1 - 1] - sx[2 * n_s + j0]};
    const double l2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double crad2 = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double q[3] = {sx[j] - T.ox - a[0], sx[n_s + j] - T.oy - a[1],
                             sx[2 * n_s + j] - T.oz - a[2]};
        double u = l2 > 0.0 ? (q[0] * b[0] + q[1] * b[1] + q[2] * b[2]) / l2 : 0.0;
        u = fmin(fmax(u, 0.0), 1.0);
        const double d[3] = {q[0] - u * b[0], q[1] - u * b[1], q[2] - u * b[2]};
        crad2 = fmax(crad2, d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
    const double margin = 1e-5 * (rad + 1.0);
    const double cm = sqrt(crad2) + nr + margin, cd = sqrt(crad2) + margin;
    T.inv_l2 = l2 > 0.0 ? (float)(1.0 / l2) : 0.0f;
    T.ax = (float)a[0];
    T.ay = (float)a[1];
    T.az = (float)a[2];
    T.bx = (float)b[0];
    T.by = (float)b[1];
    T.bz = (float)b[2];
    T.cap2_f = (float)(cm * cm) * (1.0f + 1e-6f);
    T.cap2_d = (float)(cd * cd) * (1.0f + 1e-6f);
    const double bm = (rad + band) * (1.0 + 1e-5) + 1e-30;
    T.band2_f = band > 0.0 ? (float)(bm * bm) * (1.0f + 1e-6f) : 0.0f;
    tiles[t] = T;
}

// Reductions over the 32 lanes of a half-wave (xor butterflies stay inside it).
__device__ __forceinline__ double half_min(double v) {
    for (int off = 16; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 32));
    return v;
}
__device__ __forceinline__ double half_max(double v) {
    for (int off = 16; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 32));
    return v;
}

// tile_prep_one by the 32 lanes of a half-wave, lane l taking source t * TILE + l: the
// same Tile (every quantity is a per-source expression of tile_prep_one followed by a
// min or max, which do not depend on the order), in five butterflies instead of three
// passes over the sources by one thread.  band < 0: the double layer's tangent band,
// dl_band_radius of the tile's sources with normals nrm.  Call with whole half-waves;
// every lane returns the tile.
__device__ __forceinline__ Tile tile_prep_half(int t, int l, int64_t n_s, const double* __restrict__ sx,
                                               double near_r, double near_fac,
                                               const int32_t* __restrict__ sfib, int32_t n_fib,
                                               const double* __restrict__ flen, Tile* tiles, double band,
                                               const double* __restrict__ nrm) {
    const int j0 = t * TILE;
    const int j1 = (int)min((int64_t)j0 + TILE, n_s);
    const int m = j1 - j0;
    const bool act = l < m;
    const int j = act ? j0 + l : j0;
    const double x = sx[j], y = sx[n_s + j], z = sx[2 * n_s + j];
    double lo[3], hi[3];
    lo[0] = half_min(act ? x : INFINITY);
    lo[1] = half_min(act ? y : INFINITY);
    lo[2] = half_min(act ? z : INFINITY);
    hi[0] = half_max(act ? x : -INFINITY);
    hi[1] = half_max(act ? y : -INFINITY);
    hi[2] = half_max(act ? z : -INFINITY);
    double nr = near_r;
    if (near_fac > 0.0) {
        double L = 1.0;
        if (flen) {
            int f = sfib ? sfib[j] : 0;
            if (f >= 0 && f < (sfib ? n_fib : 1)) L = flen[f];
        }
        nr = fmax(nr, half_max(act ? near_fac * L : -INFINITY));
    }
    Tile T;
    T.ox = 0.5 * (lo[0] + hi[0]);
    T.oy = 0.5 * (lo[1] + hi[1]);
    T.oz = 0.5 * (lo[2] + hi[2]);
    {
        const double dx = x - T.ox, dy = y - T.oy, dz = z - T.oz;
        const double rad2 = half_max(act ? dx * dx + dy * dy + dz * dz : 0.0);
        const double rad = sqrt(rad2);
        const double r64 = rad * (1.0 + 1e-9) + 1e-300;
        T.reach2 = r64 * r64;
        const double rm = (rad + nr) * (1.0 + 1e-5) + 1e-30;
        T.reach2_f = (float)(rm * rm) * (1.0f + 1e-6f);
        // capsule: axis from the first to the last source (lanes 0 and m - 1)
        const double x0 = __shfl(x, 0, 32), y0 = __shfl(y, 0, 32), z0 = __shfl(z, 0, 32);
        const double xe = __shfl(x, m - 1, 32), ye = __shfl(y, m - 1, 32), ze = __shfl(z, m - 1, 32);
        const double a[3] = {x0 - T.ox, y0 - T.oy, z0 - T.oz};
        const double b[3] = {xe - x0, ye - y0, ze - z0};
        const double l2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
        const double q[3] = {x - T.ox - a[0], y - T.oy - a[1], z - T.oz - a[2]};
        double u = l2 > 0.0 ? (q[0] * b[0] + q[1] * b[1] + q[2] * b[2]) / l2 : 0.0;
        u = fmin(fmax(u, 0.0), 1.0);
        const double d[3] = {q[0] - u * b[0], q[1] - u * b[1], q[2] - u * b[2]};
        const double crad2 = half_max(act ? d[0] * d[0] + d[1] * d[1] + d[2] * d[2] : 0.0);
        const double margin = 1e-5 * (rad + 1.0);
        const double cm = sqrt(crad2) + nr + margin, cd = sqrt(crad2) + margin;
        T.inv_l2 = l2 > 0.0 ? (float)(1.0 / l2) : 0.0f;
        T.ax = (float)a[0];
        T.ay = (float)a[1];
        T.az = (float)a[2];
        T.bx = (float)b[0];
        T.by = (float)b[1];
        T.bz = (float)b[2];
        T.cap2_f = (float)(cm * cm) * (1.0f + 1e-6f);
        T.cap2_d = (float)(cd * cd) * (1.0f + 1e-6f);
        if (band < 0.0) band = dl_band_radius_half(l, j0, j1, n_s, sx, nrm);
        const double bm = (rad + band) * (1.0 + 1e-5) + 1e-30;
        T.band2_f = band > 0.0 ? (float)(bm * bm) * (1.0f + 1e-6f) : 0.0f;
    }
    T.j0 = j0;
    T.j1 = j1;
    if (l == 0) tiles[t] = T;
    return T;   // the same in every lane of the half-wave
}

// Single-layer source j packed: s = pref w f, c = (eps L)^2 / 2 (0 without the
// doublet); the FP32 pack holds its position relative to its tile's FP64 origin
// (ox, oy, oz) and its near threshold.
__device__ __forceinline__ void sl_src_pack(int64_t j, int64_t n_s, const double* __restrict__ sx,
                                            const double* __restrict__ f, const double* __restrict__ w,
                                            const int32_t* __restrict__ sfib, int32_t n_fib,
                                            const double* __restrict__ flen, double pref, double eps,
                                            int doublet, double near_r, double ox, double oy, double oz,
                                            SrcSL64* s64, SrcSL32* s32, float* near_t) {
    double L = 1.0;
    if (flen) {
        const int fb = sfib ? sfib[j] : 0;
        if (fb >= 0 && fb < (sfib ? n_fib : 1)) L = flen[fb];
    }
    const double wj = w ? w[j] : 1.0;
    const double a = eps * L;
    const double c = doublet ? 0.5 * a * a : 0.0;
    SrcSL64 s;
    s.x = sx[j];
    s.y = sx[n_s + j];
    s.z = sx[2 * n_s + j];
    s.c = c;
    s.c3 = -3.0 * c;
    s.sx = pref * wj * f[j];
    s.sy = pref * wj * f[n_s + j];
    s.sz = pref * wj * f[2 * n_s + j];
    s64[j] = s;
    if (s32) {
        SrcSL32 h;
        h.x = (float)(s.x - ox);
        h.y = (float)(s.y - oy);
        h.z = (float)(s.z - oz);
        h.c = (float)c;
        h.c3 = (float)(-3.0 * c);
        h.sx = (float)s.sx;
        h.sy = (float)s.sy;
        h.sz = (float)s.sz;
        s32[j] = h;
        const double nr = fmax(near_r, 2.0 * a);
        near_t[j] = (float)(nr * nr);
    }
}

// sl_src_pack with the origin read from the tile table (tiles made earlier).
__device__ __forceinline__ void sl_src_prep_one(int64_t j, int64_t n_s, const double* __restrict__ sx,
                                                const double* __restrict__ f,
                                                const double* __restrict__ w,
                                                const int32_t* __restrict__ sfib, int32_t n_fib,
                                                const double* __restrict__ flen, double pref,
                                                double eps, int doublet, double near_r,
                                                const Tile* __restrict__ tiles, SrcSL64* s64,
                                                SrcSL32* s32, float* near_t) {
    double ox = 0.0, oy = 0.0, oz = 0.0;
    if (s32) {
        const Tile& T = tiles[j / TILE];
        ox = T.ox;
        oy = T.oy;
        oz = T.oz;
    }
    sl_src_pack(j, n_s, sx, f, w, sfib, n_fib, flen, pref, eps, doublet, near_r, ox, oy, oz, s64, s32, near_t);
}

// Double-layer source j packed: position, density q, weighted normal (3/(4 pi)) w n and
// the surface id (multi-surface sums; 0 otherwise); the FP32 pack holds its position
// relative to its tile's FP64 origin (ox, oy, oz).
__device__ __forceinline__ void dl_src_pack(int64_t j, int64_t n_s, const double* __restrict__ sx,
                                            const double* __restrict__ nrm, const double* __restrict__ w,
                                            const double* __restrict__ q, const int32_t* __restrict__ sid,
                                            double ox, double oy, double oz, SrcDL64* s64, SrcDL32* s32) {
    const double k = 3.0 / (4.0 * PI_D) * w[j];
    SrcDL64 s;
    s.x = sx[j];
    s.y = sx[n_s + j];
    s.z = sx[2 * n_s + j];
    s.qx = q[j];
    s.qy = q[n_s + j];
    s.qz = q[2 * n_s + j];
    s.nx = k * nrm[j];
    s.ny = k * nrm[n_s + j];
    s.nz = k * nrm[2 * n_s + j];
    s.pad0 = sid ? (double)sid[j] : 0.0;
    s.pad1 = s.pad2 = 0.0;
    s64[j] = s;
    if (s32) {
        SrcDL32 h;
        h.x = (float)(s.x - ox);
        h.y = (float)(s.y - oy);
        h.z = (float)(s.z - oz);
        h.qx = (float)s.qx;
        h.qy = (float)s.qy;
        h.qz = (float)s.qz;
        h.nx = (float)s.nx;
        h.ny = (float)s.ny;
        h.nz = (float)s.nz;
        h.pad0 = (float)s.pad0;
        h.pad1 = h.pad2 = 0.0f;
        s32[j] = h;
    }
}

// One block of BLOCK threads runs four waves of target block tb on chunk `chunk`.
template <int R, bool DOUBLET>
__global__ __launch_bounds__(BLOCK) void sl_fp64_kernel(SumArgs a) {
    sl_fp64_wave<R, DOUBLET>(a, blockIdx.x % a.n_tblocks, blockIdx.x / a.n_tblocks);
}
template <int R, bool DOUBLET>
__global__ __launch_bounds__(BLOCK) void sl_mixed_kernel(SumArgs a) {
    sl_mixed_wave<R, DOUBLET>(a, blockIdx.x % a.n_tblocks, blockIdx.x / a.n_tblocks);
}
template <int R, bool SUB, bool MULTI = false>
__global__ __launch_bounds__(BLOCK) void dl_fp64_kernel(SumArgs a) {
    dl_fp64_wave<R, SUB, MULTI>(a, blockIdx.x % a.n_tblocks, blockIdx.x / a.n_tblocks);
}
template <int R, bool SUB, bool MULTI = false>
__global__ __launch_bounds__(BLOCK) void dl_mixed_kernel(SumArgs a) {
    dl_mixed_wave<R, SUB, MULTI>(a, blockIdx.x % a.n_tblocks, blockIdx.x / a.n_tblocks);
}

}  // namespace stokes
