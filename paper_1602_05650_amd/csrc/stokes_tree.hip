// Far-field acceleration of the single-layer sum (the paper evaluates the sums with
// a fast multipole method, section "Matrix-vector products and FMM"): a
// kernel-independent treecode with barycentric Lagrange interpolation at
// Chebyshev points (the published method of Wang, Krasny and Tlupova, 2020),
// with the direct pair arithmetic as its near field.
//
//   Sources: a tree of boxes; every cluster C holds proxy points p_k, the tensor
//   Chebyshev points (second kind, degree n) of its box, and proxy charges
//       F_k = sum_{j in C} L_k(y_j) s_j,    D_k = sum_{j in C} L_k(y_j) c_j s_j
//   (L_k the tensor barycentric Lagrange basis of the box, s_j = w_j f_j /(8 pi mu),
//   c_j the doublet coefficient).  Targets: batches of at most 64 (median splits).
//   A batch B takes cluster C through its proxies when (r_B + r_C) < theta |c_B - c_C|
//   and C has more sources than proxies:
//       u_i += sum_k [ G(x_i - p_k) F_k + W(x_i - p_k) D_k ]   (8 pi mu G, W unscaled)
//   otherwise it recurses into C's children or, at a leaf, sums C's sources directly.
//   The error is controlled by n and theta (measured against the exact sum).
#include <math.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <type_traits>
#include <vector>

#include "pair_math.hpp"
#include "stokes_internal.hpp"
#include "tree_build.hpp"

namespace stokes {
namespace tree {

constexpr int TB = 256;        // threads per workgroup of the element-wise kernels
constexpr int MAX_DEG = 10;

// The host-side construction (clusters, batches, interaction lists) is in
// tree_build.hpp.

// ---- device kernels -------------------------------------------------------------

struct DevCl {              // what the kernels need of a proxy cluster
    double lo[3], hi[3];
    int64_t start, count;
};

// Sorted copies of a plan's points (the permutation made on the host: perm[j] is the
// input index of sorted point j) and, for plans with targets = sources, the sorted index
// of every source (inv) and of every target's own source (tself, after inv).
__global__ __launch_bounds__(TB) void k_tr_sort_src(int64_t ns, const double* xyz, const int64_t* perm, double* out,
                                                    int32_t* inv) {
    const int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (j >= ns) return;
    const int64_t o = perm[j];
    for (int c = 0; c < 3; ++c) out[c * ns + j] = xyz[c * ns + o];
    if (inv) inv[o] = (int32_t)j;
}
__global__ __launch_bounds__(TB) void k_tr_sort_trg(int64_t nt, const double* xyz, const int64_t* perm, double* out,
                                                    const int32_t* inv, int64_t* tself) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= nt) return;
    const int64_t o = perm[i];
    for (int c = 0; c < 3; ++c) out[c * nt + i] = xyz[c * nt + o];
    if (tself) tself[i] = inv[o];
}

// Sorted source packs: s = pref * w * f, doublet coefficient c = (eps L)^2 / 2 and
// the mixed path's near threshold t = max(near_r, 2 eps L)^2.
__global__ __launch_bounds__(TB) void k_tr_src(int64_t ns, const int64_t* sperm, const double* f,
                                               const double* w, const int32_t* fib, int32_t n_fib,
                                               const double* flen, double pref, double eps, double near_r,
                                               int doublet, double* ss, double* sc, float* st, int32_t* sfid) {
    const int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (j >= ns) return;
    const int64_t o = sperm[j];
    if (sfid) sfid[j] = fib[o];
    const double wj = w ? w[o] : 1.0;
    // an id outside [0, n_fib) reads no length (L = 1), as in the direct sums
    const int32_t fo = fib ? fib[o] : -1;
    const double L = (flen && fo >= 0 && fo < n_fib) ? flen[fo] : 1.0;
    const double a = eps * L;
    const double k = pref * wj;
    ss[j] = k * f[o];
    ss[ns + j] = k * f[ns + o];
    ss[2 * ns + j] = k * f[2 * ns + o];
    sc[j] = doublet ? 0.5 * a * a : 0.0;
    const double tr = fmax(near_r, 2.0 * a);
    st[j] = (float)(tr * tr);
}

// Source index range [x, y) of the fiber of every source o (fiber ids non-decreasing,
// so the range is found by two binary searches; indices stay in [0, ns] whatever the ids).
__global__ __launch_bounds__(TB) void k_tr_frange(int64_t ns, const int32_t* fib, int2* fr) {
    const int64_t o = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (o >= ns) return;
    const int32_t f = fib[o];
    int64_t lo = 0, hi = o;            // first index in [0, o] with id >= f
    while (lo < hi) {
        const int64_t m = (lo + hi) >> 1;
        if (fib[m] < f) lo = m + 1; else hi = m;
    }
    int64_t lo2 = o + 1, hi2 = ns;     // first index in [o + 1, ns) with id > f
    while (lo2 < hi2) {
        const int64_t m = (lo2 + hi2) >> 1;
        if (fib[m] <= f) lo2 = m + 1; else hi2 = m;
    }
    fr[o] = make_int2((int)lo, (int)lo2);
}

// Barycentric weights of the Chebyshev points of the second kind, cos(i pi / n)
// (the points themselves come from the plan's table, the values the proxies use).
__device__ __forceinline__ double cheb_bw(int i, int n) {
    const double s = (i & 1) ? -1.0 : 1.0;
    return (i == 0 || i == n) ? 0.5 * s : s;
}

// Proxy charges, in two steps.  Each work item is a piece of at most CH_SRC
// sources of one proxy cluster: it forms the partial charges of that piece for
// every proxy, with the 1-D barycentric basis values of SRC_TILE sources at a time
// staged in LDS.  Then k_tr_charges_sum adds each cluster's pieces in a fixed order.
// Single layer (6 per proxy): F_k = sum_j L_k(y_j) s_j, D_k = sum_j L_k(y_j) c_j s_j.
// Double layer (12): M_k = sum_j L_k(y_j) q_j (w_j n_j)^T (row-major 3 x 3),
// N_k = sum_j L_k(y_j) w_j n_j.
// A thread owns one (ky, kz) pair of the tensor grid and a group of CG charge
// components for every kx: per source it forms L_y L_z s_b once per component and
// adds L_x[kx] times it for each kx, so each LDS value feeds several FMAs.  The block
// has at least (deg + 1)^2 NC / CG threads (charges_block).
constexpr int CB = 512;            // most threads per block (degree 10, double layer: 484)
constexpr int SRC_TILE = 64;
constexpr int CG = 3;              // charge components per thread
constexpr int64_t CH_SRC = 4096;
constexpr int64_t CHARGE_ITEMS = 1024;   // aim for the number of pieces (4 per CU)
struct ChargeItem {
    int32_t q;                     // proxy slot
    int32_t count;
    int64_t start;
};
inline unsigned charges_block(int deg, int nc) {
    const int tasks = (deg + 1) * (deg + 1) * (nc / CG);
    return (unsigned)((tasks + 63) / 64 * 64);
}

// ss: [3][ns] sorted s_j (single layer) or w_j n_j (double layer); aux: [ns] c_j or
// [3][ns] q_j; xc: the deg + 1 Chebyshev points.
template <bool DL>
__global__ __launch_bounds__(CB) void k_tr_charges(int deg, const DevCl* cls, const ChargeItem* items,
                                                   const double* sxyz, int64_t ns, const double* ss,
                                                   const double* aux, const double* xc, double* part) {
    constexpr int NC = DL ? 12 : 6;
    __shared__ double lb[3][SRC_TILE][MAX_DEG + 1];
    __shared__ double sv[NC][SRC_TILE];
    const int t = threadIdx.x, nt = blockDim.x;
    const ChargeItem it = items[blockIdx.x];
    const DevCl* Cp = cls + it.q;            // (the box is indexed per thread: no private copy)
    const int n1 = deg + 1, n2 = n1 * n1, P = n2 * n1;
    const bool has = t < n2 * (NC / CG);
    const int g = t / n2, yz = t - g * n2, ky = yz / n1, kz = yz - ky * n1;
    double acc[MAX_DEG + 1][CG];
#pragma unroll
    for (int kx = 0; kx <= MAX_DEG; ++kx)
#pragma unroll
        for (int b = 0; b < CG; ++b) acc[kx][b] = 0.0;
    for (int j0 = 0; j0 < it.count; j0 += SRC_TILE) {
        const int m = min(SRC_TILE, it.count - j0);
        __syncthreads();
        for (int e = t; e < 3 * m; e += nt) {     // basis values of source jj along dimension d
            const int jj = e / 3, d = e - 3 * jj;
            const int64_t j = it.start + j0 + jj;
            const double lo = Cp->lo[d], ext = Cp->hi[d] - lo;
            const double x = 2.0 * (sxyz[d * ns + j] - lo) / ext - 1.0;
            double w[MAX_DEG + 1];
            int hit = -1;
            double den = 0.0;
#pragma unroll
            for (int i = 0; i <= MAX_DEG; ++i) {
                w[i] = 0.0;
                if (i <= deg) {
                    const double dx = x - xc[i];
                    if (dx == 0.0) hit = i;
                    w[i] = cheb_bw(i, deg) / (dx == 0.0 ? 1.0 : dx);
                    den += w[i];
                }
            }
            const double rden = 1.0 / den;
#pragma unroll
            for (int i = 0; i <= MAX_DEG; ++i)
                if (i <= deg) lb[d][jj][i] = hit >= 0 ? (i == hit ? 1.0 : 0.0) : w[i] * rden;
            if (d == 0 && !DL) {
                const double cj = aux[j];
                for (int c = 0; c < 3; ++c) {
                    sv[c][jj] = ss[c * ns + j];
                    sv[3 + c][jj] = cj * ss[c * ns + j];
                }
            }
            if (d == 0 && DL) {
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) sv[3 * r + c][jj] = aux[r * ns + j] * ss[c * ns + j];
                for (int c = 0; c < 3; ++c) sv[9 + c][jj] = ss[c * ns + j];
            }
        }
        __syncthreads();
        if (has)
            for (int jj = 0; jj < m; ++jj) {
                const double yzv = lb[1][jj][ky] * lb[2][jj][kz];
                double tv[CG];
#pragma unroll
                for (int b = 0; b < CG; ++b) tv[b] = yzv * sv[g * CG + b][jj];
#pragma unroll
                for (int kx = 0; kx <= MAX_DEG; ++kx)
                    if (kx <= deg) {
                        const double lx = lb[0][jj][kx];
#pragma unroll
                        for (int b = 0; b < CG; ++b) acc[kx][b] = fma(lx, tv[b], acc[kx][b]);
                    }
            }
    }
    if (!has) return;
    double* out = part + (int64_t)blockIdx.x * NC * P;
#pragma unroll
    for (int kx = 0; kx <= MAX_DEG; ++kx)
        if (kx <= deg)
#pragma unroll
            for (int b = 0; b < CG; ++b) out[(int64_t)(g * CG + b) * P + kx * n2 + yz] = acc[kx][b];
}

// The NC charges of every proxy cluster: its pieces summed in item order.  The first
// NA components go to pA ([n_px][NA][P]: F, or M), the others to pB (D, or N).
__global__ __launch_bounds__(TB) void k_tr_charges_sum(int P, const int32_t* item_off, const double* part,
                                                       double* pA, double* pB, int NC, int NA) {
    const int q = blockIdx.x;
    const int e = blockIdx.y * TB + threadIdx.x;   // one charge per thread
    if (e < NC * P) {
        double s = 0.0;
        for (int i = item_off[q]; i < item_off[q + 1]; ++i) s += part[(int64_t)i * NC * P + e];
        const int b = e / P, k = e - b * P;
        if (b < NA)
            pA[((int64_t)q * NA + b) * P + k] = s;
        else
            pB[((int64_t)q * (NC - NA) + b - NA) * P + k] = s;
    }
}

// FP32 charge records for the mixed evaluation, 8 floats per proxy.
__global__ __launch_bounds__(TB) void k_tr_pack(int P, const double* pF, const double* pD, float4* pk) {
    const int q = blockIdx.x;
    for (int k = threadIdx.x; k < P; k += TB) {
        const double* F = pF + (int64_t)q * 3 * P;
        const double* D = pD + (int64_t)q * 3 * P;
        pk[((int64_t)q * P + k) * 2] = make_float4((float)F[k], (float)F[P + k], (float)F[2 * P + k], (float)D[k]);
        pk[((int64_t)q * P + k) * 2 + 1] = make_float4((float)D[P + k], (float)D[2 * P + k], 0.f, 0.f);
    }
}

// FP32 charge records of the mixed double layer, 12 floats per proxy.
__global__ __launch_bounds__(TB) void k_tr_pack_dl(int P, const double* pM, const double* pN, float4* pk) {
    const int q = blockIdx.x;
    for (int k = threadIdx.x; k < P; k += TB) {
        const double* M = pM + (int64_t)q * 9 * P;
        const double* N = pN + (int64_t)q * 3 * P;
        float4* o = pk + ((int64_t)q * P + k) * 3;
        o[0] = make_float4((float)M[k], (float)M[P + k], (float)M[2 * P + k], (float)M[3 * P + k]);
        o[1] = make_float4((float)M[4 * P + k], (float)M[5 * P + k], (float)M[6 * P + k], (float)M[7 * P + k]);
        o[2] = make_float4((float)M[8 * P + k], (float)N[k], (float)N[P + k], (float)N[2 * P + k]);
    }
}

// One wave per (target batch, work part).  Lists: proxy clusters
// px_list[px_off[b] .. px_off[b+1]), direct source ranges dr_*[dr_off[b] .. dr_off[b+1]).
// A batch's entry sequence is its proxy list followed by its direct ranges; part h
// takes entries [cut[b][h], cut[b][h+1]) of it.
struct EvalArgs {
    int64_t ns, nt;
    const double* sxyz;      // [3][ns] sorted sources
    const double* ss;        // [3][ns]
    const double* sc;        // [ns]
    const float* st;         // [ns]
    const double* txyz;      // [3][nt] sorted targets
    const int64_t* tperm;    // [nt]
    const int64_t* tself;    // [nt] sorted source index of the target, or -1
    const Batch* bt;
    int32_t nb;
    const int32_t* px_off;
    const int32_t* px_list;
    const double* px_pos;    // [n_px][3][P]
    const double* pF;
    const double* pD;
    const float4* pk;        // [n_px][P][2] packed FP32 charges: F0 F1 F2 D0 | D1 D2 0 0
    const double* p1d;       // [n_px][3][deg+1] 1-D proxy coordinates of each box
    int32_t P;
    const int32_t* dr_off;
    const int64_t* dr_start;
    const int32_t* dr_count;
    int32_t S, SM;           // work parts per batch, of the SM the plan's cuts are made for
    const int32_t* cut;      // [nb][SM + 1] part boundaries in each batch's entry sequence
    double* psum;            // [S][3][nt] part sums, sorted target order
    // same-fiber exclusion (targets = sources)
    const int32_t* sfib;     // [ns] fiber id of each source, original order
    const int32_t* sfid;     // [ns] fiber id of each sorted source
    const int2* frange;      // [ns] source range of each source's fiber, original order
    const int32_t* sinv;     // [ns] sorted index of each original source
};

__device__ __forceinline__ void kahan(float& s, float& c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}


// FP64 single-layer pair (Stokeslet + doublet) into (ux, uy, uz).
// (c3 = -3 c, when the caller has it at hand)
__device__ __forceinline__ void pair64(double dx, double dy, double dz, double sx, double sy, double sz,
                                       double c, double& ux, double& uy, double& uz, double c3) {
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double ri = rsqrt64(r2);
    const double ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
    const double ds = dx * sx + dy * sy + dz * sz;
    const double A = fma(c, ri3, ri);
    const double B = ds * fma(c3, ri5, ri3);
    ux = fma(A, sx, fma(B, dx, ux));
    uy = fma(A, sy, fma(B, dy, uy));
    uz = fma(A, sz, fma(B, dz, uz));
}
__device__ __forceinline__ void pair64(double dx, double dy, double dz, double sx, double sy, double sz,
                                       double c, double& ux, double& uy, double& uz) {
    pair64(dx, dy, dz, sx, sy, sz, c, ux, uy, uz, -3.0 * c);
}

// Make the wave's LDS writes visible to all of its lanes (each wave of a workgroup
// works on its own batch and LDS region, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int EW = 4;   // waves per workgroup, each on its own (batch, part) item

// Work parts per batch for the mixed evaluation: at least 4, and more for small plans,
// up to 16, until the launch has about EVAL_WAVES waves (16 per SIMD of the 1,024).
// The FP64 evaluation, whose pairs cost about twice as much, takes twice as many
// (at most 16): the plan cuts the batches for that number, and the mixed evaluation
// uses every other cut.  (Measured on fiber sets of 32,768 to 524,288 points, degree
// 6, theta 0.7, against 2, 4, 8 and 16 parts for both.)
constexpr int64_t EVAL_WAVES = 16384;
constexpr int32_t RANGE_MOST = 512;   // sources per direct-range entry, at most
inline int eval_parts_mixed(int64_t nb) {
    int s = 4;
    while (s < 16 && s * nb < EVAL_WAVES) s *= 2;
    return s;
}
inline int eval_parts_fp64(int64_t nb) { return std::min(16, 2 * eval_parts_mixed(nb)); }

// The entry range [p_lo, p_hi) of the proxy list and [d_lo, d_hi) of the direct list
// that part h of batch b takes.
struct PartRange {
    int p_lo, p_hi, d_lo, d_hi;
};
__device__ __forceinline__ PartRange part_range(const int32_t* px_off, const int32_t* dr_off, const int32_t* cut,
                                                int S, int SM, int b, int h) {
    const int pa = px_off[b], np = px_off[b + 1] - pa, da = dr_off[b], k = SM / S;
    const int c0 = cut[(int64_t)b * (SM + 1) + h * k], c1 = cut[(int64_t)b * (SM + 1) + (h + 1) * k];
    return PartRange{pa + min(c0, np), pa + min(c1, np), da + max(c0 - np, 0), da + max(c1 - np, 0)};
}

// Sum of each target's part sums, in part order, scaled and written (or added) in the
// caller's order.  Double layer: minus half the subtracted self density (rounded to
// FP32 first on the mixed path) where q0_self is given.
__global__ __launch_bounds__(TB) void k_tr_combine(int64_t nt, int S, const double* __restrict__ psum,
                                                   const int64_t* __restrict__ tperm, double scale, double* out,
                                                   int accumulate, const int64_t* q0_self, const double* sq,
                                                   int64_t ns, int round_q0) {
    const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (i >= nt) return;
    const int64_t o = tperm[i];
    const int64_t self = q0_self ? q0_self[i] : -1;
    for (int c = 0; c < 3; ++c) {
        double r = psum[c * nt + i];
        for (int h = 1; h < S; ++h) r += psum[((int64_t)h * 3 + c) * nt + i];
        r *= scale;
        if (self >= 0) {
            double q0 = sq[c * ns + self];
            if (round_q0) q0 = (double)(float)q0;
            r -= 0.5 * q0;
        }
        if (accumulate)
            out[c * nt + o] += r;
        else
            out[c * nt + o] = r;
    }
}
// Mixed far field of one proxy cluster for a compile-time degree: the proxies form
// the tensor grid (X[kx], Y[ky], Z[kz]), so each lane keeps its z offsets and their
// squares in registers and only the six charges of a proxy come from LDS; the
// charges are staged one kx slab ((DEG+1)^2 proxies) at a time.
template <int DEG>
__device__ __forceinline__ void far_tensor(const EvalArgs& a, int q, int l, float4* slab, double cx, double cy,
                                           double cz, float xl, float yl, float zl, float& p0, float& p1,
                                           float& p2) {
    constexpr int N1 = DEG + 1, PP = N1 * N1 * N1;
    const double* X1 = a.p1d + (int64_t)q * 3 * N1;
    float DZ[N1], DZ2[N1];
#pragma unroll
    for (int kz = 0; kz < N1; ++kz) {
        DZ[kz] = zl - (float)(X1[2 * N1 + kz] - cz);
        DZ2[kz] = DZ[kz] * DZ[kz];
    }
    const float4* src = a.pk + (int64_t)q * PP * 2;
    for (int kx = 0; kx < N1; ++kx) {
        wave_sync();
        for (int e = l; e < 2 * N1 * N1; e += 64) slab[e] = src[2 * N1 * N1 * kx + e];
        wave_sync();
        const float dx = xl - (float)(X1[kx] - cx);
        const float dx2 = dx * dx;
        for (int ky = 0; ky < N1; ++ky) {
            const float dy = yl - (float)(X1[N1 + ky] - cy);
            const float rxy = fmaf(dy, dy, dx2);
#pragma unroll
            for (int kz = 0; kz < N1; ++kz) {
                const float4 f = slab[2 * (ky * N1 + kz)];
                const float4 g4 = slab[2 * (ky * N1 + kz) + 1];
                const float dz = DZ[kz];
                const float r2 = rxy + DZ2[kz];
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float ri2 = ri * ri, ri3 = ri * ri2, m3ri5 = -3.0f * (ri3 * ri2);
                const float dF = fmaf(dx, f.x, fmaf(dy, f.y, dz * f.z));
                const float dD = fmaf(dx, f.w, fmaf(dy, g4.x, dz * g4.y));
                const float g = fmaf(dD, m3ri5, dF * ri3);
                p0 = fmaf(f.x, ri, fmaf(f.w, ri3, fmaf(g, dx, p0)));
                p1 = fmaf(f.y, ri, fmaf(g4.x, ri3, fmaf(g, dy, p1)));
                p2 = fmaf(f.z, ri, fmaf(g4.y, ri3, fmaf(g, dz, p2)));
            }
        }
    }
}

// The FP64 far field of one proxy cluster on the tensor grid: z offsets and their
// squares in registers, the six FP64 charges of a proxy (F, then D) staged one kx slab
// at a time.
template <int DEG>
__device__ __forceinline__ void far_tensor64(const EvalArgs& a, int q, int l, double* slab, double cx, double cy,
                                             double cz, double xl, double yl, double zl, double& u0, double& u1,
                                             double& u2) {
    constexpr int N1 = DEG + 1, N2 = N1 * N1;
    const double* X1 = a.p1d + (int64_t)q * 3 * N1;
    const double* F = a.pF + (int64_t)q * 3 * a.P;
    const double* D = a.pD + (int64_t)q * 3 * a.P;
    double DZ[N1], DZ2[N1];
#pragma unroll
    for (int kz = 0; kz < N1; ++kz) {
        DZ[kz] = zl - (X1[2 * N1 + kz] - cz);
        DZ2[kz] = DZ[kz] * DZ[kz];
    }
    for (int kx = 0; kx < N1; ++kx) {
        wave_sync();
        for (int e = l; e < 6 * N2; e += 64) {
            const int pp = e / 6, c = e - 6 * pp, k = kx * N2 + pp;
            slab[e] = c < 3 ? F[c * a.P + k] : D[(c - 3) * a.P + k];
        }
        wave_sync();
        const double dx = xl - (X1[kx] - cx);
        const double dx2 = dx * dx;
        for (int ky = 0; ky < N1; ++ky) {
            const double dy = yl - (X1[N1 + ky] - cy);
            const double rxy = fma(dy, dy, dx2);
#pragma unroll
            for (int kz = 0; kz < N1; ++kz) {
                const double* f = slab + 6 * (ky * N1 + kz);
                const double dz = DZ[kz];
                const double r2 = rxy + DZ2[kz];
                const double ri = rsqrt64(r2);
                const double ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
                const double dF = fma(dx, f[0], fma(dy, f[1], dz * f[2]));
                const double dD = fma(dx, f[3], fma(dy, f[4], dz * f[5]));
                const double g = fma(-3.0 * dD, ri5, dF * ri3);
                u0 = fma(f[0], ri, fma(f[3], ri3, fma(g, dx, u0)));
                u1 = fma(f[1], ri, fma(f[4], ri3, fma(g, dy, u1)));
                u2 = fma(f[2], ri, fma(f[5], ri3, fma(g, dz, u2)));
            }
        }
    }
}

// (5 waves per SIMD: 96 VGPRs without spills; 6 would spill)
// EXF: same-fiber exclusion (targets = sources).  The near field skips every source of
// the target's fiber; the target's own-fiber sources that the batch took through proxy
// clusters (those in none of its direct ranges, which are sorted by start and disjoint)
// are subtracted as exact FP64 pairs, so that what remains of them is the
// interpolation error of their share of the proxy charges.  Such sources are at least
// (1 - theta) |c_B - c_C| from the target, so the subtraction is never singular.
// (the mixed EXF variant also at 5 waves: a few values spill, and it measured 2-4%
// faster than at 4; the FP64 EXF variant stays at 4)
template <bool MIXED, int DEG, bool EXF = false>
__global__ __launch_bounds__(64 * EW) __attribute__((amdgpu_waves_per_eu(EXF && !MIXED ? 4 : 5))) void k_tr_eval(EvalArgs a) {
    __shared__ __align__(16) float lfs[EW][64][12];    // (a DEG <= 8 slab: 8 (DEG+1)^2 <= 768 floats)
    __shared__ double lds_[EW][64][10];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    // wave (b, h) takes part h of batch b's entries; the parts' sums are added in part
    // order by k_tr_combine (deterministic).  The parts are cut at about equal pair
    // counts, and small plans take more of them, so that the launch fills the chip and
    // the waves of a SIMD even out.  Only wave-level synchronisation follows, so a wave
    // past the last item leaves at once.
    const int64_t gw = (int64_t)blockIdx.x * EW + w;
    const int b = (int)(gw / a.S), h = (int)(gw - (int64_t)b * a.S);
    if (b >= a.nb) return;
    const PartRange pr = part_range(a.px_off, a.dr_off, a.cut, a.S, a.SM, b, h);
    const int p_lo = pr.p_lo, p_hi = pr.p_hi, d_lo = pr.d_lo, d_hi = pr.d_hi;
    float (*lf)[12] = lfs[w];
    double (*ld)[10] = lds_[w];
    const Batch B = a.bt[b];
    const bool act = l < B.count;
    const int64_t ti = B.start + (act ? l : 0);
    const double cx = B.c[0], cy = B.c[1], cz = B.c[2];
    const double x = a.txyz[ti], y = a.txyz[a.nt + ti], z = a.txyz[2 * a.nt + ti];
    const int64_t self = a.tself ? a.tself[ti] : -1;
    const int64_t o_exf = EXF ? a.tperm[ti] : 0;
    const int32_t tf = EXF ? a.sfib[o_exf] : 0;   // the target's fiber
    const int* fidl = reinterpret_cast<const int*>(&lf[0][0]) + 8 * 64;   // after the 64 source records
    const float xl = (float)(x - cx), yl = (float)(y - cy), zl = (float)(z - cz);
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    double u0 = 0.0, u1 = 0.0, u2 = 0.0;
    // far field: proxies
    for (int e = p_lo; e < p_hi; ++e) {
        const int q = a.px_list[e];
        if constexpr (MIXED && DEG > 0) {
            float p0 = 0.f, p1 = 0.f, p2 = 0.f;
            far_tensor<DEG>(a, q, l, reinterpret_cast<float4*>(&lf[0][0]), cx, cy, cz, xl, yl, zl, p0, p1, p2);
            kahan(S0, C0, p0);
            kahan(S1, C1, p1);
            kahan(S2, C2, p2);
            continue;
        }
        if constexpr (!MIXED && DEG > 0) {
            far_tensor64<DEG>(a, q, l, &ld[0][0], cx, cy, cz, x - cx, y - cy, z - cz, u0, u1, u2);
            continue;
        }
        const double* pos = a.px_pos + (int64_t)q * 3 * a.P;
        const double* F = a.pF + (int64_t)q * 3 * a.P;
        const double* D = a.pD + (int64_t)q * 3 * a.P;
        float p0 = 0.f, p1 = 0.f, p2 = 0.f;
        for (int k0 = 0; k0 < a.P; k0 += 64) {
            const int m = min(64, a.P - k0);
            wave_sync();
            if (l < m) {
                const int k = k0 + l;
                if (MIXED) {
                    lf[l][0] = (float)(pos[k] - cx);
                    lf[l][1] = (float)(pos[a.P + k] - cy);
                    lf[l][2] = (float)(pos[2 * a.P + k] - cz);
                    for (int c = 0; c < 3; ++c) {
                        lf[l][3 + c] = (float)F[c * a.P + k];
                        lf[l][6 + c] = (float)D[c * a.P + k];
                        lf[l][9 + c] = (float)(-3.0 * D[c * a.P + k]);
                    }
                } else {
                    ld[l][0] = pos[k] - cx;
                    ld[l][1] = pos[a.P + k] - cy;
                    ld[l][2] = pos[2 * a.P + k] - cz;
                    for (int c = 0; c < 3; ++c) {
                        ld[l][3 + c] = F[c * a.P + k];
                        ld[l][6 + c] = D[c * a.P + k];
                    }
                }
            }
            wave_sync();
            if (MIXED) {
#pragma unroll 8
                for (int k = 0; k < m; ++k) {
                    const float dx = xl - lf[k][0], dy = yl - lf[k][1], dz = zl - lf[k][2];
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float ri = __builtin_amdgcn_rsqf(r2);
                    const float ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
                    const float dF = fmaf(dx, lf[k][3], fmaf(dy, lf[k][4], dz * lf[k][5]));
                    const float dD = fmaf(dx, lf[k][9], fmaf(dy, lf[k][10], dz * lf[k][11]));
                    const float g = fmaf(dD, ri5, dF * ri3);
                    p0 = fmaf(lf[k][3], ri, fmaf(lf[k][6], ri3, fmaf(g, dx, p0)));
                    p1 = fmaf(lf[k][4], ri, fmaf(lf[k][7], ri3, fmaf(g, dy, p1)));
                    p2 = fmaf(lf[k][5], ri, fmaf(lf[k][8], ri3, fmaf(g, dz, p2)));
                }
            } else {
                for (int k = 0; k < m; ++k) {
                    const double dx = (x - cx) - ld[k][0], dy = (y - cy) - ld[k][1], dz = (z - cz) - ld[k][2];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const double ri = rsqrt64(r2);
                    const double ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
                    const double dF = dx * ld[k][3] + dy * ld[k][4] + dz * ld[k][5];
                    const double dD = dx * ld[k][6] + dy * ld[k][7] + dz * ld[k][8];
                    const double g = dF * ri3 - 3.0 * dD * ri5;
                    u0 += ld[k][3] * ri + ld[k][6] * ri3 + g * dx;
                    u1 += ld[k][4] * ri + ld[k][7] * ri3 + g * dy;
                    u2 += ld[k][5] * ri + ld[k][8] * ri3 + g * dz;
                }
            }
        }
        if (MIXED) {
            kahan(S0, C0, p0);
            kahan(S1, C1, p1);
            kahan(S2, C2, p2);
        }
    }
    // EXF: the distinct fibers of the wave's targets (after the far field, whose slabs
    // share this LDS), so that a chunk of direct sources none of which lies on one of
    // them skips the per-pair fiber test
    int* fset = reinterpret_cast<int*>(&lf[0][0]) + 9 * 64;   // after the records and their fiber ids
    float* tnl = &lf[0][0] + 10 * 64;                           // the staged sources' near thresholds
    int n_fset = 0;
    if constexpr (EXF) {
        wave_sync();
        uint64_t rem = __ballot(act);
        while (rem) {   // each round takes one fiber and retires every lane on it
            const int f = __shfl(tf, __builtin_ctzll(rem));
            if (l == 0) fset[n_fset] = f;
            rem &= ~__ballot(tf == f);
            ++n_fset;
        }
        wave_sync();
    }
    // near field: direct ranges
    for (int e = d_lo; e < d_hi; ++e) {
        const int64_t j0s = a.dr_start[e];
        const int32_t cnt = a.dr_count[e];
        for (int32_t k0 = 0; k0 < cnt; k0 += 64) {
            const int m = min(64, cnt - k0);
            wave_sync();
            bool onf = false;   // EXF: this lane's source lies on one of the targets' fibers
            if (l < m) {
                const int64_t j = j0s + k0 + l;
                if (EXF) {
                    const int fj = a.sfid[j];
                    for (int i = 0; i < n_fset; ++i) onf |= fset[i] == fj;
                }
                if (MIXED) {   // records (y - c, c | s, -3 c); near thresholds apart
                    float4* r = reinterpret_cast<float4*>(&lf[0][0]) + 2 * l;
                    const float cj = (float)a.sc[j];
                    r[0] = make_float4((float)(a.sxyz[j] - cx), (float)(a.sxyz[a.ns + j] - cy),
                                       (float)(a.sxyz[2 * a.ns + j] - cz), cj);
                    r[1] = make_float4((float)a.ss[j], (float)a.ss[a.ns + j], (float)a.ss[2 * a.ns + j],
                                       -3.0f * cj);
                    tnl[l] = a.st[j];
                    if (EXF) reinterpret_cast<int*>(&lf[0][0])[8 * 64 + l] = a.sfid[j];
                } else {
                    ld[l][0] = a.sxyz[j];
                    ld[l][1] = a.sxyz[a.ns + j];
                    ld[l][2] = a.sxyz[2 * a.ns + j];
                    ld[l][3] = a.ss[j];
                    ld[l][4] = a.ss[a.ns + j];
                    ld[l][5] = a.ss[2 * a.ns + j];
                    ld[l][6] = a.sc[j];
                    if (EXF) ld[l][7] = (double)a.sfid[j];
                    ld[l][8] = -3.0 * a.sc[j];
                }
            }
            wave_sync();
            const bool fchk = EXF && __ballot(onf) != 0;   // wave-uniform
            if (MIXED) {
                float p0 = 0.f, p1 = 0.f, p2 = 0.f;
                uint64_t near = 0;
                // can any pair of this chunk be near?  Box of the staged sources (wave
                // reduction) against the batch's sphere, with the largest threshold.
                const float4* rec = reinterpret_cast<const float4*>(&lf[0][0]);
                const float4 own = rec[2 * l];
                float b0 = l < m ? own.x : INFINITY, b1 = l < m ? own.y : INFINITY,
                      b2 = l < m ? own.z : INFINITY;
                float e0 = l < m ? own.x : -INFINITY, e1 = l < m ? own.y : -INFINITY,
                      e2 = l < m ? own.z : -INFINITY, tm = l < m ? tnl[l] : 0.f;
                for (int o = 32; o > 0; o >>= 1) {
                    b0 = fminf(b0, __shfl_xor(b0, o));
                    b1 = fminf(b1, __shfl_xor(b1, o));
                    b2 = fminf(b2, __shfl_xor(b2, o));
                    e0 = fmaxf(e0, __shfl_xor(e0, o));
                    e1 = fmaxf(e1, __shfl_xor(e1, o));
                    e2 = fmaxf(e2, __shfl_xor(e2, o));
                    tm = fmaxf(tm, __shfl_xor(tm, o));
                }
                const float gx = fmaxf(0.f, fmaxf(b0, -e0)), gy = fmaxf(0.f, fmaxf(b1, -e1)),
                            gz = fmaxf(0.f, fmaxf(b2, -e2));
                const float gap = sqrtf(gx * gx + gy * gy + gz * gz) - (float)B.r;
                if (gap > 0.f && gap * gap > 1.01f * tm) {
                    // no pair can be near: the branch-free loop, with the fiber test only
                    // where a source of the chunk lies on a target's fiber
                    auto pair = [&](int k, auto fib) {
                        if constexpr (decltype(fib)::value)
                            if (fidl[k] == tf) return;
                        const float4 a0 = rec[2 * k], a1 = rec[2 * k + 1];
                        const float dx = xl - a0.x, dy = yl - a0.y, dz = zl - a0.z;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        const float ri = __builtin_amdgcn_rsqf(r2);
                        const float ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
                        const float ds = fmaf(dx, a1.x, fmaf(dy, a1.y, dz * a1.z));
                        const float A = fmaf(a0.w, ri3, ri);
                        const float Bc = ds * fmaf(a1.w, ri5, ri3);
                        p0 = fmaf(A, a1.x, fmaf(Bc, dx, p0));
                        p1 = fmaf(A, a1.y, fmaf(Bc, dy, p1));
                        p2 = fmaf(A, a1.z, fmaf(Bc, dz, p2));
                    };
                    auto far_pairs = [&](auto fib) {
                        if (m == 64) {   // a full chunk: LDS addresses are immediate offsets
#pragma unroll
                            for (int k = 0; k < 64; ++k) pair(k, fib);
                        } else {
#pragma unroll 8
                            for (int k = 0; k < m; ++k) pair(k, fib);
                        }
                    };
                    if (fchk)
                        far_pairs(std::true_type{});
                    else
                        far_pairs(std::false_type{});
                } else {
                    for (int k = 0; k < m; ++k) {
                        if (fchk && fidl[k] == tf) continue;
                        const float4 a0 = rec[2 * k], a1 = rec[2 * k + 1];
                        const float dx = xl - a0.x, dy = yl - a0.y, dz = zl - a0.z;
                        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                        if (r2 < tnl[k]) {
                            near |= 1ull << k;
                            continue;
                        }
                        const float ri = __builtin_amdgcn_rsqf(r2);
                        const float ri2 = ri * ri, ri3 = ri * ri2, ri5 = ri3 * ri2;
                        const float ds = fmaf(dx, a1.x, fmaf(dy, a1.y, dz * a1.z));
                        const float A = fmaf(a0.w, ri3, ri);
                        const float Bc = ds * fmaf(a1.w, ri5, ri3);
                        p0 = fmaf(A, a1.x, fmaf(Bc, dx, p0));
                        p1 = fmaf(A, a1.y, fmaf(Bc, dy, p1));
                        p2 = fmaf(A, a1.z, fmaf(Bc, dz, p2));
                    }
                }
                kahan(S0, C0, p0);
                kahan(S1, C1, p1);
                kahan(S2, C2, p2);
                while (near) {
                    const int k = __builtin_ctzll(near);
                    near &= near - 1;
                    const int64_t j = j0s + k0 + k;
                    if (j == self) continue;
                    const double dx = x - a.sxyz[j], dy = y - a.sxyz[a.ns + j], dz = z - a.sxyz[2 * a.ns + j];
                    if (dx == 0.0 && dy == 0.0 && dz == 0.0) continue;   // coincident: skipped
                    pair64(dx, dy, dz, a.ss[j], a.ss[a.ns + j], a.ss[2 * a.ns + j], a.sc[j], u0, u1, u2);
                }
            } else {
                // can a pair of this chunk be the target's own point or coincident?  Not
                // when the box of the staged sources lies outside the batch's sphere (FP32
                // offsets, with a margin for their rounding): then no per-pair test
                const bool in = l < m;
                float b0 = in ? (float)(ld[l][0] - cx) : INFINITY, b1 = in ? (float)(ld[l][1] - cy) : INFINITY,
                      b2 = in ? (float)(ld[l][2] - cz) : INFINITY;
                float e0 = in ? b0 : -INFINITY, e1 = in ? b1 : -INFINITY, e2 = in ? b2 : -INFINITY;
                for (int o = 32; o > 0; o >>= 1) {
                    b0 = fminf(b0, __shfl_xor(b0, o));
                    b1 = fminf(b1, __shfl_xor(b1, o));
                    b2 = fminf(b2, __shfl_xor(b2, o));
                    e0 = fmaxf(e0, __shfl_xor(e0, o));
                    e1 = fmaxf(e1, __shfl_xor(e1, o));
                    e2 = fmaxf(e2, __shfl_xor(e2, o));
                }
                const float gx = fmaxf(0.f, fmaxf(b0, -e0)), gy = fmaxf(0.f, fmaxf(b1, -e1)),
                            gz = fmaxf(0.f, fmaxf(b2, -e2));
                const float rb = (float)B.r;
                if (sqrtf(gx * gx + gy * gy + gz * gz) - rb > 1e-5f * rb) {
                    if (fchk) {
                        for (int k = 0; k < m; ++k) {
                            if (ld[k][7] == (double)tf) continue;
                            pair64(x - ld[k][0], y - ld[k][1], z - ld[k][2], ld[k][3], ld[k][4], ld[k][5], ld[k][6],
                                   u0, u1, u2, ld[k][8]);
                        }
                    } else {
#pragma unroll 4
                        for (int k = 0; k < m; ++k)
                            pair64(x - ld[k][0], y - ld[k][1], z - ld[k][2], ld[k][3], ld[k][4], ld[k][5], ld[k][6],
                                   u0, u1, u2, ld[k][8]);
                    }
                } else {
                    for (int k = 0; k < m; ++k) {
                        if (j0s + k0 + k == self) continue;
                        if (fchk && ld[k][7] == (double)tf) continue;
                        const double dx = x - ld[k][0], dy = y - ld[k][1], dz = z - ld[k][2];
                        if (dx == 0.0 && dy == 0.0 && dz == 0.0) continue;
                        pair64(dx, dy, dz, ld[k][3], ld[k][4], ld[k][5], ld[k][6], u0, u1, u2, ld[k][8]);
                    }
                }
            }
        }
    }
    if constexpr (EXF) {
        if (act) {
            const int da = a.dr_off[b], dz = a.dr_off[b + 1];   // all of the batch's direct ranges
            const int2 fr = a.frange[o_exf];
            for (int jo = fr.x + h; jo < fr.y; jo += a.S) {   // the parts take every S-th source
                const int64_t js = a.sinv[jo];
                int lo = da, hi = dz;                         // first direct range starting after js
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (a.dr_start[mid] <= js) lo = mid + 1; else hi = mid;
                }
                if (lo > da && js < a.dr_start[lo - 1] + a.dr_count[lo - 1]) continue;   // masked above
                const double ex = x - a.sxyz[js], ey = y - a.sxyz[a.ns + js], ez = z - a.sxyz[2 * a.ns + js];
                if (ex == 0.0 && ey == 0.0 && ez == 0.0) continue;
                double v0 = 0.0, v1 = 0.0, v2 = 0.0;
                pair64(ex, ey, ez, a.ss[js], a.ss[a.ns + js], a.ss[2 * a.ns + js], a.sc[js], v0, v1, v2);
                u0 -= v0;
                u1 -= v1;
                u2 -= v2;
            }
        }
    }
    double r0 = u0, r1 = u1, r2 = u2;
    if (MIXED) {
        r0 += (double)S0 - (double)C0;
        r1 += (double)S1 - (double)C1;
        r2 += (double)S2 - (double)C2;
    }
    if (!act) return;
    double* ps = a.psum + (int64_t)h * 3 * a.nt;
    ps[ti] = r0;
    ps[a.nt + ti] = r1;
    ps[2 * a.nt + ti] = r2;
}

// ---- double layer ---------------------------------------------------------------
// u_i = (3 / (4 pi)) sum_{s != self} (d . (q_s - q0))(d . w_s n_s) d / |d|^5 - q0 / 2
// (d = x_i - y_s; q0 = q_self on the surface with subtraction, else 0 and no -q0/2).
// On a proxy p_k the sum over its cluster's sources becomes
// (d^T M_k d - (d . q0)(d . N_k)) d / |d|^5, d = x_i - p_k.

// Sorted double-layer sources: wn = w n, q.
__global__ __launch_bounds__(TB) void k_tr_dlsrc(int64_t ns, const int64_t* sperm, const double* n,
                                                 const double* w, const double* q, double* wn, double* sq) {
    const int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (j >= ns) return;
    const int64_t o = sperm[j];
    const double wj = w[o];
    for (int c = 0; c < 3; ++c) {
        wn[c * ns + j] = wj * n[c * ns + o];
        sq[c * ns + j] = q[c * ns + o];
    }
}

// Mixed double layer: per sorted source, the squared radius below which its direct pairs
// are taken in FP64: the larger of the near radius and the tangent band of the source's
// run of 32 sorted sources (dl_band_radius; the sort keeps a run spatially compact).
__global__ __launch_bounds__(TB) void k_tr_dlband(int64_t ns, const double* __restrict__ sxyz,
                                                  const double* __restrict__ wn, double near_r, float* st) {
    const int64_t j = (int64_t)blockIdx.x * TB + threadIdx.x;
    if (j >= ns) return;
    const int64_t j0 = j & ~(int64_t)31, j1 = j0 + 32 < ns ? j0 + 32 : ns;
    const double r = fmax(near_r, dl_band_radius<false>(j0, j1, ns, sxyz, wn));
    st[j] = (float)(r * r);
}

struct DlArgs {
    int64_t ns, nt;
    const double* sxyz;      // [3][ns] sorted sources
    const double* wn;        // [3][ns] w n
    const double* sq;        // [3][ns] q
    const double* txyz;      // [3][nt] sorted targets
    const int64_t* tperm;
    const int64_t* tself;    // [nt] sorted source index of the target, or null (off the surface)
    const Batch* bt;
    int32_t nb;
    const int32_t* px_off;
    const int32_t* px_list;
    const double* px_pos;    // [n_px][3][P]
    const double* pM;        // [n_px][9][P]
    const double* pN;        // [n_px][3][P]
    const float4* pk;        // mixed: [n_px][P][3] FP32 charges M0..M3 | M4..M7 | M8 N0 N1 N2
    const double* p1d;       // [n_px][3][deg+1] 1-D proxy coordinates of each box
    int32_t P;
    const int32_t* dr_off;
    const int64_t* dr_start;
    const int32_t* dr_count;
    int32_t S, SM;           // as in EvalArgs
    const int32_t* cut;
    double* psum;
    int subtract;
    const float* near2;      // mixed: [ns] FP64 below this squared distance (k_tr_dlband)
};

// Mixed double-layer far field of one proxy cluster for a compile-time degree, on the
// tensor grid as far_tensor: the lane keeps its z offsets and their squares in
// registers, the twelve FP32 charges of a proxy come from LDS one kx slab at a time,
// and the slab's sum takes one Kahan step.
template <int DEG>
__device__ __forceinline__ void far_tensor_dl(const DlArgs& a, int q, int l, float4* slab, double cx, double cy,
                                              double cz, float xl, float yl, float zl, float fq0x, float fq0y,
                                              float fq0z, float& S0, float& S1, float& S2, float& C0, float& C1,
                                              float& C2) {
    constexpr int N1 = DEG + 1, N2 = N1 * N1;
    const double* X1 = a.p1d + (int64_t)q * 3 * N1;
    float DZ[N1], DZ2[N1];
#pragma unroll
    for (int kz = 0; kz < N1; ++kz) {
        DZ[kz] = zl - (float)(X1[2 * N1 + kz] - cz);
        DZ2[kz] = DZ[kz] * DZ[kz];
    }
    const float4* src = a.pk + (int64_t)q * N2 * N1 * 3;
    for (int kx = 0; kx < N1; ++kx) {
        wave_sync();
        for (int e = l; e < 3 * N2; e += 64) slab[e] = src[3 * N2 * kx + e];
        wave_sync();
        const float dx = xl - (float)(X1[kx] - cx);
        const float dx2 = dx * dx;
        float p0 = 0.f, p1 = 0.f, p2 = 0.f;
        for (int ky = 0; ky < N1; ++ky) {
            const float dy = yl - (float)(X1[N1 + ky] - cy);
            const float rxy = fmaf(dy, dy, dx2);
            const float qxy = fmaf(dx, fq0x, dy * fq0y);
#pragma unroll
            for (int kz = 0; kz < N1; ++kz) {
                const float4 f0 = slab[3 * (ky * N1 + kz)], f1 = slab[3 * (ky * N1 + kz) + 1],
                             f2 = slab[3 * (ky * N1 + kz) + 2];
                const float dz = DZ[kz];
                const float r2 = rxy + DZ2[kz];
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float m0 = fmaf(f0.x, dx, fmaf(f0.y, dy, f0.z * dz));
                const float m1 = fmaf(f0.w, dx, fmaf(f1.x, dy, f1.y * dz));
                const float m2 = fmaf(f1.z, dx, fmaf(f1.w, dy, f2.x * dz));
                const float dMd = fmaf(dx, m0, fmaf(dy, m1, dz * m2));
                const float dN = fmaf(dx, f2.y, fmaf(dy, f2.z, dz * f2.w));
                const float dq0 = fmaf(dz, fq0z, qxy);
                const float kk = fmaf(-dq0, dN, dMd) * rinv5_f32(r2, ri);
                p0 = fmaf(kk, dx, p0);
                p1 = fmaf(kk, dy, p1);
                p2 = fmaf(kk, dz, p2);
            }
        }
        kahan(S0, C0, p0);
        kahan(S1, C1, p1);
        kahan(S2, C2, p2);
    }
}

// The FP64 double-layer far field of one proxy cluster on the tensor grid: z offsets
// and their squares in registers, the twelve FP64 charges of a proxy (M row-major,
// then N) staged one kx slab at a time.
template <int DEG>
__device__ __forceinline__ void far_tensor_dl64(const DlArgs& a, int q, int l, double* slab, double cx, double cy,
                                                double cz, double xl, double yl, double zl, double q0x, double q0y,
                                                double q0z, double& u0, double& u1, double& u2) {
    constexpr int N1 = DEG + 1, N2 = N1 * N1;
    const double* X1 = a.p1d + (int64_t)q * 3 * N1;
    const double* M = a.pM + (int64_t)q * 9 * a.P;
    const double* Nn = a.pN + (int64_t)q * 3 * a.P;
    double DZ[N1], DZ2[N1];
#pragma unroll
    for (int kz = 0; kz < N1; ++kz) {
        DZ[kz] = zl - (X1[2 * N1 + kz] - cz);
        DZ2[kz] = DZ[kz] * DZ[kz];
    }
    for (int kx = 0; kx < N1; ++kx) {
        wave_sync();
        for (int e = l; e < 12 * N2; e += 64) {
            const int pp = e / 12, c = e - 12 * pp, k = kx * N2 + pp;
            slab[e] = c < 9 ? M[c * a.P + k] : Nn[(c - 9) * a.P + k];
        }
        wave_sync();
        const double dx = xl - (X1[kx] - cx);
        const double dx2 = dx * dx;
        for (int ky = 0; ky < N1; ++ky) {
            const double dy = yl - (X1[N1 + ky] - cy);
            const double rxy = fma(dy, dy, dx2);
            const double qxy = fma(dx, q0x, dy * q0y);
#pragma unroll
            for (int kz = 0; kz < N1; ++kz) {
                const double* f = slab + 12 * (ky * N1 + kz);
                const double dz = DZ[kz];
                const double r2 = rxy + DZ2[kz];
                const double ri = rsqrt64(r2);
                const double ri2 = ri * ri, ri5 = ri2 * ri2 * ri;
                const double m0 = fma(f[0], dx, fma(f[1], dy, f[2] * dz));
                const double m1 = fma(f[3], dx, fma(f[4], dy, f[5] * dz));
                const double m2 = fma(f[6], dx, fma(f[7], dy, f[8] * dz));
                const double dMd = fma(dx, m0, fma(dy, m1, dz * m2));
                const double dN = fma(dx, f[9], fma(dy, f[10], dz * f[11]));
                const double dq0 = fma(dz, q0z, qxy);
                const double kk = fma(-dq0, dN, dMd) * ri5;
                u0 = fma(kk, dx, u0);
                u1 = fma(kk, dy, u1);
                u2 = fma(kk, dz, u2);
            }
        }
    }
}

// Wave (b, h) takes part h of batch b's proxy and direct lists, as in k_tr_eval; the
// parts' sums are added in part order, scaled and completed by k_tr_combine.  MIXED: proxies and direct pairs in
// FP32 relative to the batch centre, each cluster's or chunk's sum added with Kahan
// compensation; direct pairs closer than the source's near2 (the near radius or the
// tangent band, and the self point) are taken in FP64 from the sorted sources.  The
// subtracted self density is rounded to FP32 once and used as such everywhere (FP32
// pairs and proxies, FP64 pairs, jump term), so that its constant part cancels against
// the jump up to the discrete identity's defect.
template <bool MIXED, int DEG = 0>
__global__ __launch_bounds__(64 * EW) __attribute__((amdgpu_waves_per_eu(MIXED && DEG > 0 ? 4 : 1))) void k_tr_dl_eval(DlArgs a) {
    __shared__ double lds_[EW][64][16];   // (an FP64 slab of degree <= 8: 12 (DEG+1)^2 <= 972 doubles)
    __shared__ float lfs[EW][64][16];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * EW + w;
    const int b = (int)(gw / a.S), h = (int)(gw - (int64_t)b * a.S);
    if (b >= a.nb) return;
    const PartRange pr = part_range(a.px_off, a.dr_off, a.cut, a.S, a.SM, b, h);
    const int p_lo = pr.p_lo, p_hi = pr.p_hi, d_lo = pr.d_lo, d_hi = pr.d_hi;
    double (*ld)[16] = lds_[w];
    const Batch B = a.bt[b];
    const bool act = l < B.count;
    const int64_t ti = B.start + (act ? l : 0);
    const double cx = B.c[0], cy = B.c[1], cz = B.c[2];
    const double x = a.txyz[ti], y = a.txyz[a.nt + ti], z = a.txyz[2 * a.nt + ti];
    const double xl = x - cx, yl = y - cy, zl = z - cz;
    const int64_t self = a.tself ? a.tself[ti] : -1;
    const bool sub = a.subtract && self >= 0;
    double q0x = sub ? a.sq[self] : 0.0, q0y = sub ? a.sq[a.ns + self] : 0.0,
           q0z = sub ? a.sq[2 * a.ns + self] : 0.0;
    if (MIXED) {
        q0x = (double)(float)q0x;
        q0y = (double)(float)q0y;
        q0z = (double)(float)q0z;
    }
    double u0 = 0.0, u1 = 0.0, u2 = 0.0;
    float (*lf)[16] = lfs[w];
    const float fxl = (float)xl, fyl = (float)yl, fzl = (float)zl;
    const float fq0x = (float)q0x, fq0y = (float)q0y, fq0z = (float)q0z;
    float S0 = 0.f, S1 = 0.f, S2 = 0.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    // far field: proxies
    for (int e = p_lo; e < p_hi; ++e) {
        const int q = a.px_list[e];
        const double* pos = a.px_pos + (int64_t)q * 3 * a.P;
        const double* M = a.pM + (int64_t)q * 9 * a.P;
        const double* N = a.pN + (int64_t)q * 3 * a.P;
        if constexpr (MIXED && DEG > 0) {
            far_tensor_dl<DEG>(a, q, l, reinterpret_cast<float4*>(&lf[0][0]), cx, cy, cz, fxl, fyl, fzl, fq0x, fq0y,
                               fq0z, S0, S1, S2, C0, C1, C2);
            continue;
        }
        if constexpr (!MIXED && DEG > 0) {
            far_tensor_dl64<DEG>(a, q, l, &ld[0][0], cx, cy, cz, xl, yl, zl, q0x, q0y, q0z, u0, u1, u2);
            continue;
        }
        if constexpr (MIXED) {
            for (int k0 = 0; k0 < a.P; k0 += 64) {     // Kahan step per 64 proxies
                const int m = min(64, a.P - k0);
                float p0 = 0.f, p1 = 0.f, p2 = 0.f;
                wave_sync();
                if (l < m) {
                    const int k = k0 + l;
                    lf[l][0] = (float)(pos[k] - cx);
                    lf[l][1] = (float)(pos[a.P + k] - cy);
                    lf[l][2] = (float)(pos[2 * a.P + k] - cz);
                    for (int c = 0; c < 9; ++c) lf[l][3 + c] = (float)M[c * a.P + k];
                    for (int c = 0; c < 3; ++c) lf[l][12 + c] = (float)N[c * a.P + k];
                }
                wave_sync();
#pragma unroll 4
                for (int k = 0; k < m; ++k) {
                    const float dx = fxl - lf[k][0], dy = fyl - lf[k][1], dz = fzl - lf[k][2];
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float ri = __builtin_amdgcn_rsqf(r2);
                    const float m0 = fmaf(lf[k][3], dx, fmaf(lf[k][4], dy, lf[k][5] * dz));
                    const float m1 = fmaf(lf[k][6], dx, fmaf(lf[k][7], dy, lf[k][8] * dz));
                    const float m2 = fmaf(lf[k][9], dx, fmaf(lf[k][10], dy, lf[k][11] * dz));
                    const float dMd = fmaf(dx, m0, fmaf(dy, m1, dz * m2));
                    const float dN = fmaf(dx, lf[k][12], fmaf(dy, lf[k][13], dz * lf[k][14]));
                    const float dq0 = fmaf(dx, fq0x, fmaf(dy, fq0y, dz * fq0z));
                    const float kk = fmaf(-dq0, dN, dMd) * rinv5_f32(r2, ri);
                    p0 = fmaf(kk, dx, p0);
                    p1 = fmaf(kk, dy, p1);
                    p2 = fmaf(kk, dz, p2);
                }
                kahan(S0, C0, p0);
                kahan(S1, C1, p1);
                kahan(S2, C2, p2);
            }
            continue;
        }
        for (int k0 = 0; k0 < a.P; k0 += 64) {
            const int m = min(64, a.P - k0);
            wave_sync();
            if (l < m) {
                const int k = k0 + l;
                ld[l][0] = pos[k] - cx;
                ld[l][1] = pos[a.P + k] - cy;
                ld[l][2] = pos[2 * a.P + k] - cz;
                for (int c = 0; c < 9; ++c) ld[l][3 + c] = M[c * a.P + k];
                for (int c = 0; c < 3; ++c) ld[l][12 + c] = N[c * a.P + k];
            }
            wave_sync();
            for (int k = 0; k < m; ++k) {
                const double dx = xl - ld[k][0], dy = yl - ld[k][1], dz = zl - ld[k][2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double ri = rsqrt64(r2);
                const double ri2 = ri * ri, ri5 = ri2 * ri2 * ri;
                const double m0 = ld[k][3] * dx + ld[k][4] * dy + ld[k][5] * dz;
                const double m1 = ld[k][6] * dx + ld[k][7] * dy + ld[k][8] * dz;
                const double m2 = ld[k][9] * dx + ld[k][10] * dy + ld[k][11] * dz;
                const double dMd = dx * m0 + dy * m1 + dz * m2;
                const double dN = dx * ld[k][12] + dy * ld[k][13] + dz * ld[k][14];
                const double dq0 = dx * q0x + dy * q0y + dz * q0z;
                const double kk = (dMd - dq0 * dN) * ri5;
                u0 += kk * dx;
                u1 += kk * dy;
                u2 += kk * dz;
            }
        }
    }
    // near field: direct ranges
    for (int e = d_lo; e < d_hi; ++e) {
        const int64_t j0s = a.dr_start[e];
        const int32_t cnt = a.dr_count[e];
        for (int32_t k0 = 0; k0 < cnt; k0 += 64) {
            const int m = min(64, cnt - k0);
            if constexpr (MIXED) {
                wave_sync();
                if (l < m) {
                    const int64_t j = j0s + k0 + l;
                    lf[l][0] = (float)(a.sxyz[j] - cx);
                    lf[l][1] = (float)(a.sxyz[a.ns + j] - cy);
                    lf[l][2] = (float)(a.sxyz[2 * a.ns + j] - cz);
                    for (int c = 0; c < 3; ++c) {
                        lf[l][3 + c] = (float)a.wn[c * a.ns + j];
                        lf[l][6 + c] = (float)a.sq[c * a.ns + j];
                    }
                    lf[l][9] = a.near2[j];
                }
                wave_sync();
                float p0 = 0.f, p1 = 0.f, p2 = 0.f;
                uint64_t near = 0;
#pragma unroll 4
                for (int k = 0; k < m; ++k) {
                    const float dx = fxl - lf[k][0], dy = fyl - lf[k][1], dz = fzl - lf[k][2];
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    if (r2 < lf[k][9]) {                // includes the self point
                        near |= 1ull << k;
                        continue;
                    }
                    const float ri = __builtin_amdgcn_rsqf(r2);
                    const float dq = fmaf(dx, lf[k][6] - fq0x, fmaf(dy, lf[k][7] - fq0y, dz * (lf[k][8] - fq0z)));
                    const float dn = fmaf(dx, lf[k][3], fmaf(dy, lf[k][4], dz * lf[k][5]));
                    const float kk = dq * dn * rinv5_f32(r2, ri);
                    p0 = fmaf(kk, dx, p0);
                    p1 = fmaf(kk, dy, p1);
                    p2 = fmaf(kk, dz, p2);
                }
                kahan(S0, C0, p0);
                kahan(S1, C1, p1);
                kahan(S2, C2, p2);
                while (near) {
                    const int k = __builtin_ctzll(near);
                    near &= near - 1;
                    const int64_t j = j0s + k0 + k;
                    if (j == self) continue;
                    const double dx = x - a.sxyz[j], dy = y - a.sxyz[a.ns + j], dz = z - a.sxyz[2 * a.ns + j];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 == 0.0) continue;                    // coincident: skipped
                    const double ri = rsqrt64(r2), ri2 = ri * ri;
                    const double dq = dx * (a.sq[j] - q0x) + dy * (a.sq[a.ns + j] - q0y) +
                                      dz * (a.sq[2 * a.ns + j] - q0z);
                    const double dn = dx * a.wn[j] + dy * a.wn[a.ns + j] + dz * a.wn[2 * a.ns + j];
                    const double kk = dq * dn * (ri2 * ri2 * ri);
                    u0 += kk * dx;
                    u1 += kk * dy;
                    u2 += kk * dz;
                }
                continue;
            }
            wave_sync();
            if (l < m) {
                const int64_t j = j0s + k0 + l;
                for (int c = 0; c < 3; ++c) {
                    ld[l][c] = a.sxyz[c * a.ns + j];
                    ld[l][3 + c] = a.wn[c * a.ns + j];
                    ld[l][6 + c] = a.sq[c * a.ns + j];
                }
            }
            wave_sync();
            for (int k = 0; k < m; ++k) {
                if (j0s + k0 + k == self) continue;
                const double dx = x - ld[k][0], dy = y - ld[k][1], dz = z - ld[k][2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;                            // coincident: skipped
                const double ri = rsqrt64(r2), ri2 = ri * ri;
                const double dq = dx * (ld[k][6] - q0x) + dy * (ld[k][7] - q0y) + dz * (ld[k][8] - q0z);
                const double dn = dx * ld[k][3] + dy * ld[k][4] + dz * ld[k][5];
                const double kk = dq * dn * (ri2 * ri2 * ri);
                u0 += kk * dx;
                u1 += kk * dy;
                u2 += kk * dz;
            }
        }
    }
    if (MIXED) {
        u0 += (double)S0 - (double)C0;
        u1 += (double)S1 - (double)C1;
        u2 += (double)S2 - (double)C2;
    }
    if (!act) return;
    double* ps = a.psum + (int64_t)h * 3 * a.nt;
    ps[ti] = u0;
    ps[a.nt + ti] = u1;
    ps[2 * a.nt + ti] = u2;
}

}  // namespace tree
}  // namespace stokes

using namespace stokes;
using namespace stokes::tree;

struct stokes_tree {
    int64_t ns = 0, nt = 0;
    bool same = false;
    int deg = 0, P = 0;
    double theta = 0.0;
    int32_t nb = 0, n_px = 0;
    int64_t pairs_px = 0, pairs_dir = 0;
    void* mem = nullptr;
    // device views into mem
    double* sxyz = nullptr;
    int64_t* sperm = nullptr;
    double* txyz = nullptr;
    int64_t* tperm = nullptr;
    int64_t* tself = nullptr;
    Batch* bt = nullptr;
    int32_t* px_off = nullptr;
    int32_t* px_list = nullptr;
    DevCl* px_cl = nullptr;
    double* px_pos = nullptr;
    double* pF = nullptr;
    double* pD = nullptr;
    double* pM = nullptr;
    double* pN = nullptr;
    int32_t* dr_off = nullptr;
    int64_t* dr_start = nullptr;
    int32_t* dr_count = nullptr;
    double* ss = nullptr;
    double* sc = nullptr;
    float* st = nullptr;
    double* sq = nullptr;         // [3][ns] sorted double-layer density
    float4* pk = nullptr;
    double* p1d = nullptr;
    int32_t* sinv = nullptr;      // targets = sources only: sorted index of each source,
    int32_t* sfid = nullptr;      // fiber id of each sorted source and
    int2* frange = nullptr;       // the source range of each source's fiber (filled per evaluation)
    int32_t n_items = 0;
    ChargeItem* items = nullptr;
    int32_t* item_off = nullptr;
    double* part = nullptr;
    int32_t S_mix = 4, S = 8;     // evaluation work parts per batch: mixed, FP64 (the cuts' own)
    int32_t* cut = nullptr;       // [nb][S + 1]
    double* psum = nullptr;       // [S][3][nt]
    double* xc = nullptr;         // [deg + 1] Chebyshev points cos(i pi / deg)
    ~stokes_tree() {
        if (mem) (void)hipFree(mem);
    }
};

extern "C" int stokes_tree_create(int64_t n_src, const double* src_xyz, int64_t n_trg,
                                  const double* trg_xyz, int32_t degree, double theta,
                                  int32_t leaf_size, void* stream, stokes_tree** out) {
    if (!out) return fail(STOKES_E_INVAL, "stokes_tree_create: null out");
    *out = nullptr;
    if (n_src < 1 || !src_xyz) return fail(STOKES_E_INVAL, "stokes_tree_create: need n_src >= 1 and src_xyz");
    if (degree < 1 || degree > MAX_DEG) return fail(STOKES_E_INVAL, "stokes_tree_create: degree must be 1..10");
    if (!(theta > 0.0 && theta < 1.0)) return fail(STOKES_E_INVAL, "stokes_tree_create: theta must be in (0, 1)");
    if (leaf_size < 1) return fail(STOKES_E_INVAL, "stokes_tree_create: leaf_size must be >= 1");
    const bool same = trg_xyz == nullptr;
    if (same) n_trg = n_src;
    if (n_trg < 1) return fail(STOKES_E_INVAL, "stokes_tree_create: need n_trg >= 1");
    if (n_src >= ((int64_t)1 << 31) || n_trg >= ((int64_t)1 << 31))
        return fail(STOKES_E_INVAL, "stokes_tree_create: too many points");
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<double> hs(3 * n_src), ht;
    STOKES_HIP(hipMemcpyAsync(hs.data(), src_xyz, 3 * n_src * 8, hipMemcpyDeviceToHost, st));
    if (!same) {
        ht.resize(3 * n_trg);
        STOKES_HIP(hipMemcpyAsync(ht.data(), trg_xyz, 3 * n_trg * 8, hipMemcpyDeviceToHost, st));
    }
    STOKES_HIP(hipStreamSynchronize(st));
    for (double v : hs)
        if (!std::isfinite(v)) return fail(STOKES_E_NONFINITE, "stokes_tree_create: non-finite source position");
    for (double v : ht)
        if (!std::isfinite(v)) return fail(STOKES_E_NONFINITE, "stokes_tree_create: non-finite target position");
    const std::vector<double>& tx = same ? hs : ht;

    std::vector<int64_t> sperm, tperm;
    std::vector<Cluster> cl;
    std::vector<Batch> bt;
    // the source tree and the target batches are independent: built side by side
    std::thread batches([&] { build_batches(tx, n_trg, tperm, bt, plan_threads(n_trg)); });
    build_sources(hs, n_src, sperm, cl, leaf_size, plan_threads(n_src));
    batches.join();
    const int n1 = degree + 1, P = n1 * n1 * n1;
    Lists lists;
    build_lists(bt, cl, theta, P, lists, plan_threads(n_trg));
    split_ranges(lists, RANGE_MOST);
    const std::vector<int32_t>& px_off = lists.px_off;
    const std::vector<int32_t>& px_list = lists.px_list;
    const std::vector<int32_t>& used = lists.used;
    const std::vector<int32_t>& dr_off = lists.dr_off;
    const std::vector<int64_t>& dr_start = lists.dr_start;
    const std::vector<int32_t>& dr_count = lists.dr_count;
    const int64_t pairs_px = lists.pairs_px, pairs_dir = lists.pairs_dir;
    // proxy clusters: boxes (degenerate extents padded) and Chebyshev points
    std::vector<double> cheb(n1);   // cos(i pi / n), the second-kind points on [-1, 1]
    for (int i = 0; i < n1; ++i) cheb[i] = std::cos(i * 3.14159265358979323846 / degree);
    const int32_t n_px = (int32_t)used.size();
    std::vector<DevCl> pcl(n_px);
    std::vector<double> ppos((size_t)n_px * 3 * P);
    for (int32_t q = 0; q < n_px; ++q) {
        const Cluster& C = cl[used[q]];
        double emax = 0.0;
        for (int d = 0; d < 3; ++d) emax = std::max(emax, C.hi[d] - C.lo[d]);
        for (int d = 0; d < 3; ++d) {
            double lo = C.lo[d], hi = C.hi[d];
            const double minext = emax > 0.0 ? 1e-3 * emax : 1.0;   // flat or point-like boxes
            if (hi - lo < minext) {
                const double m = 0.5 * (lo + hi);
                lo = m - 0.5 * minext;
                hi = m + 0.5 * minext;
            }
            pcl[q].lo[d] = lo;
            pcl[q].hi[d] = hi;
        }
        pcl[q].start = C.start;
        pcl[q].count = C.count;
        for (int k = 0; k < P; ++k) {
            const int idx[3] = {k / (n1 * n1), (k / n1) % n1, k % n1};
            for (int d = 0; d < 3; ++d)
                ppos[((size_t)q * 3 + d) * P + k] =
                    pcl[q].lo[d] + 0.5 * (cheb[idx[d]] + 1.0) * (pcl[q].hi[d] - pcl[q].lo[d]);
        }
    }
    // 1-D proxy coordinates of each box: [q][dim][i] = lo + (1 + cos(i pi / n)) (hi - lo) / 2
    std::vector<double> p1d((size_t)n_px * 3 * n1);
    for (int32_t q = 0; q < n_px; ++q)
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < n1; ++i)
                p1d[((size_t)q * 3 + d) * n1 + i] =
                    pcl[q].lo[d] + 0.5 * (cheb[i] + 1.0) * (pcl[q].hi[d] - pcl[q].lo[d]);
    // charge work items: pieces of each proxy cluster's sources, about CHARGE_ITEMS of
    // them in all (whole LDS tiles, at most CH_SRC sources)
    int64_t px_src = 0;
    for (int32_t q = 0; q < n_px; ++q) px_src += pcl[q].count;
    const int64_t ch = std::min<int64_t>(
        CH_SRC, std::max<int64_t>(1, (px_src + CHARGE_ITEMS * SRC_TILE - 1) / (CHARGE_ITEMS * SRC_TILE)) * SRC_TILE);
    std::vector<ChargeItem> items;
    std::vector<int32_t> item_off{0};
    for (int32_t q = 0; q < n_px; ++q) {
        for (int64_t o = 0; o < pcl[q].count; o += ch)
            items.push_back(ChargeItem{q, (int32_t)std::min<int64_t>(ch, pcl[q].count - o), pcl[q].start + o});
        item_off.push_back((int32_t)items.size());
    }
    // evaluation work parts: S per batch, cut at about equal pair counts
    const int64_t nb = (int64_t)bt.size();
    const int S = eval_parts_fp64(nb);
    const std::vector<int32_t> cut = part_cuts(lists, P, S);
    // (the sorted coordinates and the self indices are made on the device, k_tr_sort_*)
    const size_t n_inv = same ? (size_t)n_src : 0, n_self = same ? (size_t)n_trg : 0;

    // one device allocation
    auto t = new stokes_tree();
    t->ns = n_src;
    t->nt = n_trg;
    t->same = same;
    t->deg = degree;
    t->P = P;
    t->theta = theta;
    t->nb = (int32_t)bt.size();
    t->n_px = n_px;
    t->pairs_px = pairs_px;
    t->pairs_dir = pairs_dir;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (std::max<size_t>(bytes, 8) + 255) & ~size_t(255);
        return o;
    };
    const size_t o_sx = take(3 * n_src * 8), o_sp = take(n_src * 8), o_tx = take(3 * n_trg * 8),
                 o_tp = take(n_trg * 8), o_ts = take(n_self * 8), o_bt = take(bt.size() * sizeof(Batch)),
                 o_po = take(px_off.size() * 4), o_pl = take(px_list.size() * 4),
                 o_pc = take((size_t)n_px * sizeof(DevCl)), o_pp = take(ppos.size() * 8),
                 o_pF = take(ppos.size() * 4 * 8), o_do = take(dr_off.size() * 4),
                 o_ds = take(dr_start.size() * 8), o_dc = take(dr_count.size() * 4), o_ss = take(3 * n_src * 8),
                 o_sc = take(n_src * 8), o_st = take(n_src * 4), o_it = take(items.size() * sizeof(ChargeItem)),
                 o_io = take(item_off.size() * 4), o_pa = take(items.size() * 12 * P * 8),
                 o_sq = take(3 * n_src * 8),
                 o_pk = take((size_t)n_px * P * 48), o_p1 = take(p1d.size() * 8),
                 o_si = take(n_inv * 4), o_sf = take(n_inv * 4), o_fr = take(n_inv * 8),
                 o_cu = take(cut.size() * 4), o_ps = take((size_t)S * 3 * n_trg * 8), o_xc = take(cheb.size() * 8);
    hipError_t e = hipMalloc(&t->mem, off);
    if (e != hipSuccess) {
        delete t;
        return hip_fail(e, "hipMalloc(tree)");
    }
    char* base = static_cast<char*>(t->mem);
    t->sxyz = reinterpret_cast<double*>(base + o_sx);
    t->sperm = reinterpret_cast<int64_t*>(base + o_sp);
    t->txyz = reinterpret_cast<double*>(base + o_tx);
    t->tperm = reinterpret_cast<int64_t*>(base + o_tp);
    t->tself = same ? reinterpret_cast<int64_t*>(base + o_ts) : nullptr;
    t->bt = reinterpret_cast<Batch*>(base + o_bt);
    t->px_off = reinterpret_cast<int32_t*>(base + o_po);
    t->px_list = reinterpret_cast<int32_t*>(base + o_pl);
    t->px_cl = reinterpret_cast<DevCl*>(base + o_pc);
    t->px_pos = reinterpret_cast<double*>(base + o_pp);
    t->pF = reinterpret_cast<double*>(base + o_pF);
    // proxy charges, 12 P doubles per cluster: single layer F [n_px][3][P] then
    // D [n_px][3][P]; double layer M [n_px][9][P] then N [n_px][3][P]
    t->pD = t->pF + ppos.size();
    t->pM = t->pF;
    t->pN = t->pF + 3 * ppos.size();
    t->sq = reinterpret_cast<double*>(base + o_sq);
    t->dr_off = reinterpret_cast<int32_t*>(base + o_do);
    t->dr_start = reinterpret_cast<int64_t*>(base + o_ds);
    t->dr_count = reinterpret_cast<int32_t*>(base + o_dc);
    t->ss = reinterpret_cast<double*>(base + o_ss);
    t->sc = reinterpret_cast<double*>(base + o_sc);
    t->st = reinterpret_cast<float*>(base + o_st);
    t->n_items = (int32_t)items.size();
    t->items = reinterpret_cast<ChargeItem*>(base + o_it);
    t->item_off = reinterpret_cast<int32_t*>(base + o_io);
    t->part = reinterpret_cast<double*>(base + o_pa);
    t->pk = reinterpret_cast<float4*>(base + o_pk);
    t->p1d = reinterpret_cast<double*>(base + o_p1);
    t->S = S;
    t->S_mix = eval_parts_mixed(nb);
    t->cut = reinterpret_cast<int32_t*>(base + o_cu);
    t->psum = reinterpret_cast<double*>(base + o_ps);
    t->xc = reinterpret_cast<double*>(base + o_xc);
    if (same) {
        t->sinv = reinterpret_cast<int32_t*>(base + o_si);
        t->sfid = reinterpret_cast<int32_t*>(base + o_sf);
        t->frange = reinterpret_cast<int2*>(base + o_fr);
    }
    auto up = [&](void* dst, const void* src, size_t bytes) -> int {
        if (!bytes) return STOKES_OK;
        hipError_t r = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
        return r == hipSuccess ? STOKES_OK : hip_fail(r, "hipMemcpyAsync(tree)");
    };
    int rc = STOKES_OK;
    if (!rc) rc = up(t->sperm, sperm.data(), n_src * 8);
    if (!rc) rc = up(t->tperm, tperm.data(), n_trg * 8);
    if (!rc) {   // sorted coordinates; the inverse source permutation before the self indices
        hipLaunchKernelGGL(k_tr_sort_src, dim3((unsigned)((n_src + TB - 1) / TB)), dim3(TB), 0, st, n_src, src_xyz,
                           (const int64_t*)t->sperm, t->sxyz, t->sinv);
        hipLaunchKernelGGL(k_tr_sort_trg, dim3((unsigned)((n_trg + TB - 1) / TB)), dim3(TB), 0, st, n_trg,
                           same ? src_xyz : trg_xyz, (const int64_t*)t->tperm, t->txyz, (const int32_t*)t->sinv,
                           t->tself);
        const hipError_t r = hipGetLastError();
        if (r != hipSuccess) rc = hip_fail(r, "tree sort kernels");
    }
    if (!rc) rc = up(t->bt, bt.data(), bt.size() * sizeof(Batch));
    if (!rc) rc = up(t->px_off, px_off.data(), px_off.size() * 4);
    if (!rc) rc = up(t->px_list, px_list.data(), px_list.size() * 4);
    if (!rc) rc = up(t->px_cl, pcl.data(), pcl.size() * sizeof(DevCl));
    if (!rc) rc = up(t->px_pos, ppos.data(), ppos.size() * 8);
    if (!rc) rc = up(t->dr_off, dr_off.data(), dr_off.size() * 4);
    if (!rc) rc = up(t->dr_start, dr_start.data(), dr_start.size() * 8);
    if (!rc) rc = up(t->dr_count, dr_count.data(), dr_count.size() * 4);
    if (!rc) rc = up(t->items, items.data(), items.size() * sizeof(ChargeItem));
    if (!rc) rc = up(t->item_off, item_off.data(), item_off.size() * 4);
    if (!rc) rc = up(t->p1d, p1d.data(), p1d.size() * 8);
    if (!rc) rc = up(t->cut, cut.data(), cut.size() * 4);
    if (!rc) rc = up(t->xc, cheb.data(), cheb.size() * 8);
    if (!rc) {
        hipError_t r = hipStreamSynchronize(st);
        if (r != hipSuccess) rc = hip_fail(r, "hipStreamSynchronize(tree)");
    }
    if (rc) {
        delete t;
        return rc;
    }
    *out = t;
    return STOKES_OK;
}

template <bool EXF>
static void launch_eval(bool mixed, int deg, unsigned grid, dim3 blk, hipStream_t st, const EvalArgs& a) {
    if (!mixed) {
        switch (deg) {
            case 4: hipLaunchKernelGGL((k_tr_eval<false, 4, EXF>), dim3(grid), blk, 0, st, a); break;
            case 5: hipLaunchKernelGGL((k_tr_eval<false, 5, EXF>), dim3(grid), blk, 0, st, a); break;
            case 6: hipLaunchKernelGGL((k_tr_eval<false, 6, EXF>), dim3(grid), blk, 0, st, a); break;
            case 7: hipLaunchKernelGGL((k_tr_eval<false, 7, EXF>), dim3(grid), blk, 0, st, a); break;
            case 8: hipLaunchKernelGGL((k_tr_eval<false, 8, EXF>), dim3(grid), blk, 0, st, a); break;
            default: hipLaunchKernelGGL((k_tr_eval<false, 0, EXF>), dim3(grid), blk, 0, st, a); break;
        }
        return;
    }
    switch (deg) {   // the tensor-grid far field for the common degrees
        case 4: hipLaunchKernelGGL((k_tr_eval<true, 4, EXF>), dim3(grid), blk, 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_tr_eval<true, 5, EXF>), dim3(grid), blk, 0, st, a); break;
        case 6: hipLaunchKernelGGL((k_tr_eval<true, 6, EXF>), dim3(grid), blk, 0, st, a); break;
        case 7: hipLaunchKernelGGL((k_tr_eval<true, 7, EXF>), dim3(grid), blk, 0, st, a); break;
        case 8: hipLaunchKernelGGL((k_tr_eval<true, 8, EXF>), dim3(grid), blk, 0, st, a); break;
        default: hipLaunchKernelGGL((k_tr_eval<true, 0, EXF>), dim3(grid), blk, 0, st, a); break;
    }
}

extern "C" int stokes_tree_sl_eval(stokes_tree* t, const double* src_force, const double* src_weight,
                                   const int32_t* src_fiber, int32_t n_fib, const double* fiber_len,
                                   double mu, double eps, double near_r, uint32_t flags, double* u_out,
                                   void* stream) {
    if (!t) return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: null tree");
    if (flags & ~(STOKES_PREC_MIXED | STOKES_EXCL_SELF_POINT | STOKES_EXCL_SAME_FIBER | STOKES_NO_DOUBLET |
                  STOKES_ACCUMULATE | STOKES_CHECK_INPUTS))
        return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: unsupported flag bits");
    if (src_fiber && n_fib < 1) return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: src_fiber needs n_fib >= 1");
    if (!std::isfinite(near_r)) return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: near_r not finite");
    const bool exf = flags & STOKES_EXCL_SAME_FIBER;
    if (exf && (flags & STOKES_EXCL_SELF_POINT))
        return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: choose one exclusion mode");
    if ((flags & (STOKES_EXCL_SELF_POINT | STOKES_EXCL_SAME_FIBER)) && !t->same)
        return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: exclusion needs targets = sources");
    if (!src_force || !u_out) return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: null pointer");
    if ((src_fiber == nullptr) != (fiber_len == nullptr))
        return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: src_fiber and fiber_len go together");
    if (exf && !src_fiber) return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: same-fiber exclusion needs src_fiber");
    if (!(mu > 0.0)) return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: mu must be > 0");
    if (!(eps > 0.0 && eps < 0.5)) return fail(STOKES_E_INVAL, "stokes_tree_sl_eval: eps must be in (0, 0.5)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (flags & STOKES_CHECK_INPUTS) {   // the direct sums' scan (synchronous)
        if (int rc = scan_sl_inputs(st, "stokes_tree_sl_eval", t->ns, src_force, src_weight, src_fiber, n_fib,
                                    fiber_len))
            return rc;
    }
    const bool mixed = flags & STOKES_PREC_MIXED;
    const double pref = 1.0 / (8.0 * 3.14159265358979323846 * mu);
    hipLaunchKernelGGL(k_tr_src, dim3((unsigned)((t->ns + TB - 1) / TB)), dim3(TB), 0, st, t->ns, t->sperm,
                       src_force, src_weight, src_fiber, src_fiber ? n_fib : 0, fiber_len, pref, eps, near_r,
                       (flags & STOKES_NO_DOUBLET) ? 0 : 1, t->ss, t->sc, t->st, exf ? t->sfid : nullptr);
    if (exf)
        hipLaunchKernelGGL(k_tr_frange, dim3((unsigned)((t->ns + TB - 1) / TB)), dim3(TB), 0, st, t->ns, src_fiber,
                           t->frange);
    if (t->n_px > 0) {
        hipLaunchKernelGGL(k_tr_charges<false>, dim3(t->n_items), dim3(charges_block(t->deg, 6)), 0, st, t->deg,
                           (const DevCl*)t->px_cl, (const ChargeItem*)t->items, (const double*)t->sxyz, t->ns,
                           (const double*)t->ss, (const double*)t->sc, (const double*)t->xc, t->part);
        hipLaunchKernelGGL(k_tr_charges_sum, dim3(t->n_px, (6 * t->P + TB - 1) / TB), dim3(TB), 0, st, t->P,
                           (const int32_t*)t->item_off, (const double*)t->part, t->pF, t->pD, 6, 3);
        if (mixed)
            hipLaunchKernelGGL(k_tr_pack, dim3(t->n_px), dim3(TB), 0, st, t->P, (const double*)t->pF,
                               (const double*)t->pD, t->pk);
    }
    EvalArgs a{};
    a.ns = t->ns;
    a.nt = t->nt;
    a.sxyz = t->sxyz;
    a.ss = t->ss;
    a.sc = t->sc;
    a.st = t->st;
    a.txyz = t->txyz;
    a.tperm = t->tperm;
    a.tself = (flags & STOKES_EXCL_SELF_POINT) ? t->tself : nullptr;
    a.bt = t->bt;
    a.nb = t->nb;
    a.px_off = t->px_off;
    a.px_list = t->px_list;
    a.px_pos = t->px_pos;
    a.pF = t->pF;
    a.pD = t->pD;
    a.pk = t->pk;
    a.p1d = t->p1d;
    a.P = t->P;
    a.dr_off = t->dr_off;
    a.dr_start = t->dr_start;
    a.dr_count = t->dr_count;
    a.S = mixed ? t->S_mix : t->S;
    a.SM = t->S;
    a.cut = t->cut;
    a.psum = t->psum;
    a.sfib = src_fiber;
    a.sfid = t->sfid;
    a.frange = t->frange;
    a.sinv = t->sinv;
    const unsigned grid = (unsigned)(((int64_t)t->nb * a.S + EW - 1) / EW);
    const dim3 blk(64 * EW);
    if (exf)
        launch_eval<true>(mixed, t->deg, grid, blk, st, a);
    else
        launch_eval<false>(mixed, t->deg, grid, blk, st, a);
    hipLaunchKernelGGL(k_tr_combine, dim3((unsigned)((t->nt + TB - 1) / TB)), dim3(TB), 0, st, t->nt, a.S,
                       (const double*)t->psum, (const int64_t*)t->tperm, 1.0, u_out,
                       (flags & STOKES_ACCUMULATE) ? 1 : 0, (const int64_t*)nullptr, (const double*)nullptr,
                       t->ns, 0);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

extern "C" int stokes_tree_dl_eval(stokes_tree* t, const double* src_normal, const double* src_weight,
                                   const double* src_q, double near_r, uint32_t flags, double* u_out,
                                   void* stream) {
    if (!t) return fail(STOKES_E_INVAL, "stokes_tree_dl_eval: null tree");
    if (!std::isfinite(near_r)) return fail(STOKES_E_INVAL, "stokes_tree_dl_eval: near_r not finite");
    if (flags & ~(STOKES_PREC_MIXED | STOKES_ONSURF_RAW | STOKES_ACCUMULATE))
        return fail(STOKES_E_INVAL, "stokes_tree_dl_eval: unsupported flag bits");
    if (!src_normal || !src_weight || !src_q || !u_out)
        return fail(STOKES_E_INVAL, "stokes_tree_dl_eval: null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_tr_dlsrc, dim3((unsigned)((t->ns + TB - 1) / TB)), dim3(TB), 0, st, t->ns, t->sperm,
                       src_normal, src_weight, src_q, t->ss, t->sq);
    if (t->n_px > 0) {
        hipLaunchKernelGGL(k_tr_charges<true>, dim3(t->n_items), dim3(charges_block(t->deg, 12)), 0, st, t->deg,
                           (const DevCl*)t->px_cl, (const ChargeItem*)t->items, (const double*)t->sxyz, t->ns,
                           (const double*)t->ss, (const double*)t->sq, (const double*)t->xc, t->part);
        hipLaunchKernelGGL(k_tr_charges_sum, dim3(t->n_px, (12 * t->P + TB - 1) / TB), dim3(TB), 0, st, t->P,
                           (const int32_t*)t->item_off, (const double*)t->part, t->pM, t->pN, 12, 9);
        if (flags & STOKES_PREC_MIXED)
            hipLaunchKernelGGL(k_tr_pack_dl, dim3(t->n_px), dim3(TB), 0, st, t->P, (const double*)t->pM,
                               (const double*)t->pN, t->pk);
    }
    DlArgs a{};
    a.ns = t->ns;
    a.nt = t->nt;
    a.sxyz = t->sxyz;
    a.wn = t->ss;
    a.sq = t->sq;
    a.txyz = t->txyz;
    a.tperm = t->tperm;
    a.tself = t->same ? t->tself : nullptr;
    a.bt = t->bt;
    a.nb = t->nb;
    a.px_off = t->px_off;
    a.px_list = t->px_list;
    a.px_pos = t->px_pos;
    a.pM = t->pM;
    a.pN = t->pN;
    a.pk = t->pk;
    a.p1d = t->p1d;
    a.P = t->P;
    a.dr_off = t->dr_off;
    a.dr_start = t->dr_start;
    a.dr_count = t->dr_count;
    a.S = (flags & STOKES_PREC_MIXED) ? t->S_mix : t->S;
    a.SM = t->S;
    a.cut = t->cut;
    a.psum = t->psum;
    a.subtract = (flags & STOKES_ONSURF_RAW) ? 0 : 1;
    const double nr = near_r > 0.0 ? near_r : 0.02;
    if (flags & STOKES_PREC_MIXED)
        hipLaunchKernelGGL(k_tr_dlband, dim3((unsigned)((t->ns + TB - 1) / TB)), dim3(TB), 0, st, t->ns,
                           (const double*)t->sxyz, (const double*)t->ss, nr, t->st);
    a.near2 = t->st;
    const unsigned grid = (unsigned)(((int64_t)t->nb * a.S + EW - 1) / EW);
    if (!(flags & STOKES_PREC_MIXED)) {
        switch (t->deg) {   // the tensor-grid far field for the common degrees
            case 4: hipLaunchKernelGGL((k_tr_dl_eval<false, 4>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            case 5: hipLaunchKernelGGL((k_tr_dl_eval<false, 5>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            case 6: hipLaunchKernelGGL((k_tr_dl_eval<false, 6>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            case 7: hipLaunchKernelGGL((k_tr_dl_eval<false, 7>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            case 8: hipLaunchKernelGGL((k_tr_dl_eval<false, 8>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            default: hipLaunchKernelGGL((k_tr_dl_eval<false, 0>), dim3(grid), dim3(64 * EW), 0, st, a); break;
        }
    } else {
        switch (t->deg) {   // the tensor-grid far field for the common degrees
            case 4: hipLaunchKernelGGL((k_tr_dl_eval<true, 4>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            case 5: hipLaunchKernelGGL((k_tr_dl_eval<true, 5>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            case 6: hipLaunchKernelGGL((k_tr_dl_eval<true, 6>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            case 7: hipLaunchKernelGGL((k_tr_dl_eval<true, 7>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            case 8: hipLaunchKernelGGL((k_tr_dl_eval<true, 8>), dim3(grid), dim3(64 * EW), 0, st, a); break;
            default: hipLaunchKernelGGL((k_tr_dl_eval<true, 0>), dim3(grid), dim3(64 * EW), 0, st, a); break;
        }
    }
    const double pref = 3.0 / (4.0 * 3.14159265358979323846);
    hipLaunchKernelGGL(k_tr_combine, dim3((unsigned)((t->nt + TB - 1) / TB)), dim3(TB), 0, st, t->nt, a.S,
                       (const double*)t->psum, (const int64_t*)t->tperm, pref, u_out,
                       (flags & STOKES_ACCUMULATE) ? 1 : 0,
                       (const int64_t*)(t->same && a.subtract ? t->tself : nullptr), (const double*)t->sq, t->ns,
                       (flags & STOKES_PREC_MIXED) ? 1 : 0);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

namespace stokes {
int FarPlan::make(int64_t n, const double* xyz, const stokes_far& far, hipStream_t st) {
    if (far.degree < 1 || far.degree > tree::MAX_DEG || !(far.theta > 0.0 && far.theta < 1.0))
        return fail(STOKES_E_INVAL, "stokes_far: degree must be 1..10 and theta in (0, 1)");
    return stokes_tree_create(n, xyz, 0, nullptr, far.degree, far.theta, far.leaf_size > 0 ? far.leaf_size : 128,
                              st, &t);
}
}  // namespace stokes

extern "C" int stokes_tree_info(const stokes_tree* t, int64_t* proxy_pairs, int64_t* direct_pairs,
                                int32_t* n_proxy_clusters, int32_t* n_batches) {
    if (!t) return fail(STOKES_E_INVAL, "stokes_tree_info: null tree");
    if (proxy_pairs) *proxy_pairs = t->pairs_px;
    if (direct_pairs) *direct_pairs = t->pairs_dir;
    if (n_proxy_clusters) *n_proxy_clusters = t->n_px;
    if (n_batches) *n_batches = t->nb;
    return STOKES_OK;
}

extern "C" int stokes_tree_destroy(stokes_tree* t) {
    if (!t) return fail(STOKES_E_INVAL, "stokes_tree_destroy: null tree");
    delete t;
    return STOKES_OK;
}
