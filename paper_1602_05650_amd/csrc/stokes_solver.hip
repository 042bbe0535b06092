// Fiber mobility solve: right-preconditioned GMRES in FP64 on the device.
//
//   A f = M f [+ K_delta f] + u_bar[f] = V    (eq. main-sb-local; K_delta the
//                                       regularised nonlocal self term of
//                                       eq. sb-stokes-reg; u_bar from all other
//                                       fibers, eq. complementary-uf)
//   P = M (the local 3x3 node blocks) or, block-Jacobi (section "Linear solver
//       and preconditioner"), each fiber's self block M [+ K_delta], inverted
//       once per request by Gauss-Jordan elimination
//   GMRES (Saad) on A P^{-1} y = V from y0 = 0: Arnoldi with classical
//   Gram-Schmidt applied twice, Givens rotations, x = P^{-1} V_m y.
//
// Every kernel here works on a batch of requests (see solver_batch.hpp).
#include <math.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "fiber_device.hpp"
#include "gj_device.hpp"
#include "solver_batch.hpp"

namespace stokes {

constexpr int G_ELEM = 512;   // grid of the elementwise kernels in graph mode
constexpr int G_SL = 2048;    // grid of the single-layer kernel in graph mode
constexpr int G_ONE = MAX_SLOTS;

__device__ __forceinline__ int find_slot(cptr<WorkList> wl, int64_t item) {
    int lo = 0, hi = wl->n - 1;
    while (lo < hi) {   // largest s with prefix[s] <= item
        const int mid = (lo + hi + 1) >> 1;
        if (wl->prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// (B_f^{-1} v) at node i of fiber f: rows c npf + kk of the fiber's inverse block
// (column-major, m = 3 npf) against the fiber's 3 npf values of v.
__device__ __forceinline__ void block_apply(const double* binv, int64_t i, int64_t N, int npf,
                                            const double* v, double& ox, double& oy,
                                            double& oz) {
    const int f = (int)(i / npf), kk = (int)(i % npf), m = 3 * npf;
    const double* A = binv + (int64_t)f * m * m;
    const int64_t f0 = (int64_t)f * npf;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int col = 0; col < m; ++col) {
        const int e = col / npf, k = col - e * npf;
        const double vc = v[(int64_t)e * N + f0 + k];
        const double* Ac = A + (int64_t)col * m + kk;
        a0 = fma(Ac[0], vc, a0);
        a1 = fma(Ac[npf], vc, a1);
        a2 = fma(Ac[2 * npf], vc, a2);
    }
    ox = a0;
    oy = a1;
    oz = a2;
}

// Partial dot products of m vectors A[i] (stride) with w.  A slot's dot work items are
// B element blocks times dot_groups(k) groups of DOT_GROUP vectors: item `item` covers
// block b = item % B of the elements and vectors [i0, i0 + DOT_GROUP) with
// i0 = DOT_GROUP (item / B), so the groups of one iteration run in parallel (a group
// at or past m has nothing to do).  Per vector the order of the arithmetic is fixed:
// each thread's strided partial over block b, then a fixed tree.
constexpr int DOT_GROUP = 8;
__host__ __device__ inline int dot_groups(int k) { return (k + DOT_GROUP) / DOT_GROUP; }   // covers m <= k + 1
__device__ void dot_partials(const double* A, int64_t stride, int m, const double* w, int64_t n,
                             int B, int item, double* out, double (*lds)[BLOCK]) {
    const int b = item % B;
    const int i0 = (item / B) * DOT_GROUP;
    if (i0 >= m) return;   // block-uniform
    const int64_t L = (n + B - 1) / B;
    const int64_t e0 = (int64_t)b * L;
    const int64_t e1 = min(n, e0 + L);
    const int t = threadIdx.x;
    const int g_n = min(DOT_GROUP, m - i0);
    double s[DOT_GROUP];
#pragma unroll
    for (int g = 0; g < DOT_GROUP; ++g) s[g] = 0.0;
    for (int64_t e = e0 + t; e < e1; e += BLOCK) {
        const double we = w[e];
#pragma unroll
        for (int g = 0; g < DOT_GROUP; ++g)
            if (g < g_n) s[g] = fma(A[(int64_t)(i0 + g) * stride + e], we, s[g]);
    }
#pragma unroll
    for (int g = 0; g < DOT_GROUP; ++g) lds[g][t] = s[g];
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (t < h) {
#pragma unroll
            for (int g = 0; g < DOT_GROUP; ++g) lds[g][t] += lds[g][t + h];
        }
        __syncthreads();
    }
    if (t < g_n) out[(int64_t)(i0 + t) * B + b] = lds[t][0];
    __syncthreads();
}

// ---- set-up kernels (eager, at admission) ------------------------------------
__global__ __launch_bounds__(BLOCK) void k_geom(const SlotDesc* D, const StepTables* T) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_PRE];
    const int64_t total = wl->prefix[wl->n];
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int64_t i = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (i < d.N) {
            const int f = (int)(i / d.npf);
            const int kk = (int)(i % d.npf);
            d.fib[i] = f;
            d.wq[i] = cc_weight(kk, d.npf - 1) * 0.5 * d.flen[f];
            d.sarc[i] = 0.5 * d.flen[f] * (1.0 + cos(kk * 3.14159265358979323846 / (d.npf - 1)));
            d.excl[i] = make_int2(f * d.npf, f * d.npf + d.npf);
        }
    }
}

// Bounding spheres of the source tiles (after k_geom: reads the fiber ids).
__global__ __launch_bounds__(BLOCK) void k_tiles(const SlotDesc* D, const StepTables* T) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_PRE];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int64_t t = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (t < d.sl.n_tiles)
            tile_prep_one((int)t, d.N, d.xyz, d.near_r, d.sl.s32 ? 2.0 * d.eps : 0.0, d.fib,
                          d.n_fib, d.flen, d.tiles);
    }
}

// Self block M [+ K_delta] of one fiber (after k_geom), inverted by Gauss-Jordan
// elimination with partial pivoting (gj_device.hpp): one workgroup of BLOCK_GJ
// threads per fiber holds the m x m matrix (m = 3 npf) in registers.  The inverse
// is written column-major to the slot's binv buffer (row and column index c npf + k).
__global__ __launch_bounds__(BLOCK_GJ) void k_block(const SlotDesc* D, const StepTables* T) {
    __shared__ GjLds sh;
    const cptr<WorkList> wl = &as_const(T)->wl[WL_FIB];
    const int t = threadIdx.x;
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int f = (int)(it - wl->prefix[si]);
        const int npf = d.npf, m = 3 * npf;
        const int64_t N = d.N, f0 = (int64_t)f * npf;
        const bool nl = d.opts & STOKES_NONLOCAL;
        const double d2 = d.delta * d.delta;
        const bool act = t < GJ_G * m;
        const int r = act ? t % m : 0, g = act ? t / m : 0;   // as gj_invert expects
        const int rc = r / npf, ri = r - rc * npf;
        const int64_t gi = f0 + ri;
        // this row's node: position, tangent, and the subtracted K_delta coefficient
        const double xi = d.xyz[gi], yi = d.xyz[N + gi], zi = d.xyz[2 * N + gi];
        const double rti = d.tan[rc * N + gi];
        double dsum = 0.0;
        if (nl)
            for (int q = 0; q < npf; ++q) {
                if (q == ri) continue;
                const double ds = d.sarc[gi] - d.sarc[f0 + q];
                dsum += d.wq[f0 + q] / sqrt(ds * ds + d2);
            }
        double A[GJ_COLS];
#pragma unroll
        for (int jj = 0; jj < GJ_COLS; ++jj) {
            const int c = g + GJ_G * jj;
            double v = 0.0;
            if (act && c < m) {
                const int ce = c / npf, k = c - ce * npf;
                const double id = rc == ce ? 1.0 : 0.0;
                if (k != ri) {
                    if (nl) {
                        const int64_t gk = f0 + k;
                        const double rx = xi - d.xyz[gk], ry = yi - d.xyz[N + gk], rz = zi - d.xyz[2 * N + gk];
                        const double r2 = rx * rx + ry * ry + rz * rz;
                        const double ra = rc == 0 ? rx : (rc == 1 ? ry : rz);
                        const double rb = ce == 0 ? rx : (ce == 1 ? ry : rz);
                        v = d.pref * d.wq[gk] * (id + ra * rb / r2) / sqrt(r2 + d2);
                    }
                } else {
                    const double te = d.tan[ce * N + gi];
                    v = d.pref * ((d.kappa + 2.0) * id + (d.kappa - 2.0) * rti * te);
                    if (nl) v -= d.pref * dsum * (id + rti * te);
                }
            }
            A[jj] = v;
        }
        gj_invert(m, act, r, g, A, sh, d.binv + (int64_t)f * m * m);
        __syncthreads();
    }
}

// beta = |rhs| partials (WL_DOT), then beta and v_0 (WL_ONE, WL_VEC).
__global__ __launch_bounds__(BLOCK) void k_init_norm(const SlotDesc* D, const StepTables* T) {
    __shared__ double lds[DOT_GROUP][BLOCK];
    const cptr<WorkList> wl = &as_const(T)->wl[WL_DOT];
    const int64_t total = wl->prefix[wl->n];
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        dot_partials(d.rhs, 0, 1, d.rhs, 3 * (int64_t)d.N, d.B, (int)(it - wl->prefix[si]), d.normp,
                     lds);
    }
}

__global__ __launch_bounds__(BLOCK) void k_init_beta(const SlotDesc* D, const StepTables* T,
                                                     double* stat) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_ONE];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const auto& d = as_const(D)[wl->slot[find_slot(wl, it)]];
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int b = 0; b < d.B; ++b) s += d.normp[b];
            const double beta = sqrt(s);
            d.g[0] = beta;
            for (int i = 1; i <= d.k; ++i) d.g[i] = 0.0;
            double* st = stat + NSTAT * d.sid;
            st[0] = 0.0;
            st[1] = beta;
            st[2] = beta;
            st[3] = beta == 0.0 ? 1.0 : 0.0;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_init_v0(const SlotDesc* D, const StepTables* T) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_VEC];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int64_t e = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (e < 3 * (int64_t)d.N) {
            const double beta = d.g[0];
            d.V[e] = beta > 0.0 ? d.rhs[e] / beta : 0.0;
        }
    }
}

// ---- step kernels ------------------------------------------------------------------
// z = P^{-1} v_j and the packed single-layer sources s = pref * wq * z.
__global__ __launch_bounds__(BLOCK) void k_pre(const SlotDesc* D, const StepTables* T, int doublet) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_PRE];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int64_t i = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (i >= d.N) continue;
        const int64_t N = d.N;
        const double* v = d.V + (int64_t)d.j * 3 * N;
        double fx, fy, fz;
        if (d.opts & STOKES_PRECOND_BLOCK) {
            block_apply(d.binv, i, N, d.npf, v, fx, fy, fz);
        } else {
            fx = v[i];
            fy = v[N + i];
            fz = v[2 * N + i];
            apply_local(d.kappa, d.mu, true, d.tan[i], d.tan[N + i], d.tan[2 * N + i], fx, fy, fz);
        }
        d.z[i] = fx;
        d.z[N + i] = fy;
        d.z[2 * N + i] = fz;
        if (!(d.opts & OPT_FAR))   // a far slot's sum is the treecode's
            sl_src_prep_one(i, N, d.xyz, d.z, d.wq, d.fib, d.n_fib, d.flen, d.pref, d.eps, doublet,
                            d.near_r, d.tiles, d.s64, d.s32, d.near_t);
    }
}

template <bool MIXED, bool DOUBLET>
__global__ __launch_bounds__(BLOCK) void k_sl(const SlotDesc* D, const StepTables* T) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_SL];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        // copy the slot's sum arguments into registers with scalar loads
        SumArgs a;
        {
            static_assert(sizeof(SumArgs) % 8 == 0, "SumArgs is copied in 8-byte words");
            const cptr<uint64_t> w = (cptr<uint64_t>)&as_const(D)[wl->slot[si]].sl;
            uint64_t* o = reinterpret_cast<uint64_t*>(&a);
#pragma unroll
            for (int q = 0; q < (int)(sizeof(SumArgs) / 8); ++q) o[q] = w[q];
        }
        const int local = (int)(wl->base[si] + (it - wl->prefix[si]));
        const int tb = local % a.n_tblocks;
        const int chunk = local / a.n_tblocks;
        if (MIXED)
            sl_mixed_wave<R_SL32, DOUBLET>(a, tb, chunk);
        else
            sl_fp64_wave<R_SL64, DOUBLET>(a, tb, chunk);
    }
}

// w = M z + (sum of the chunk partials, in chunk order).
__global__ __launch_bounds__(BLOCK) void k_red(const SlotDesc* D, const StepTables* T) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_RED];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int64_t i = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (i >= d.N) continue;
        const int64_t N = d.N;
        double u[3] = {0.0, 0.0, 0.0};
        const int nch = d.n_items_sl / d.sl.n_tblocks;
        for (int k = 0; k < nch; ++k) {
            const double* p = d.partial + (int64_t)k * 3 * N;
            u[0] += p[i];
            u[1] += p[N + i];
            u[2] += p[2 * N + i];
        }
        double mx = d.z[i], my = d.z[N + i], mz = d.z[2 * N + i];
        apply_local(d.kappa, d.mu, false, d.tan[i], d.tan[N + i], d.tan[2 * N + i], mx, my, mz);
        if (d.opts & STOKES_NONLOCAL) {
            double kx, ky, kz;
            nonlocal_at(i, N, d.npf, d.xyz, d.tan, d.z, d.wq, d.sarc, d.delta, d.pref, kx, ky, kz);
            mx += kx;
            my += ky;
            mz += kz;
        }
        d.w[i] = mx + u[0];
        d.w[N + i] = my + u[1];
        d.w[2 * N + i] = mz + u[2];
    }
}

// which = 0: partials of V[0..j].w ; which = 1: same (second Gram-Schmidt pass);
// which = 2: partials of w.w (norm).
__global__ __launch_bounds__(BLOCK) void k_dot(const SlotDesc* D, const StepTables* T, int which) {
    __shared__ double lds[DOT_GROUP][BLOCK];
    const cptr<WorkList> wl = &as_const(T)->wl[WL_DOT];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int b = (int)(it - wl->prefix[si]);
        const int64_t n = 3 * (int64_t)d.N;
        if (which == 2)
            dot_partials(d.w, 0, 1, d.w, n, d.B, b, d.normp, lds);
        else
            dot_partials(d.V, n, d.j + 1, d.w, n, d.B, b, d.dotp, lds);
    }
}

// hs[i] = the sum over b < B of p[i B + b], for i < m, by the whole block: tpr threads
// per row (8, 16 or 32: more when there are fewer rows; thread t takes row i0 + t / tpr
// and the partials b = t % tpr, t % tpr + tpr, ... in order, four loads ahead), then a
// fixed butterfly over the tpr threads, which leaves the same value in each of them.
// The caller synchronises before reading hs.
__device__ void block_sum_rows(const double* p, int B, int m, double* hs) {
    const int tpr = m > 16 ? 8 : (m > 8 ? 16 : 32);
    const int r = threadIdx.x / tpr, q = threadIdx.x % tpr;
    for (int i0 = 0; i0 < m; i0 += BLOCK / tpr) {
        const int i = i0 + r;
        double s = 0.0;
        if (i < m) {
            const double* pr = p + (int64_t)i * B;
            int b = q;
            for (; b + 3 * tpr < B; b += 4 * tpr) {
                const double a0 = pr[b], a1 = pr[b + tpr], a2 = pr[b + 2 * tpr], a3 = pr[b + 3 * tpr];
                s += a0;
                s += a1;
                s += a2;
                s += a3;
            }
            for (; b < B; b += tpr) s += pr[b];
        }
        for (int o = tpr / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (i < m && q == 0) hs[i] = s;
    }
}

// w -= sum_i V[i] h[i] (i ascending) with h[i] = the sum of the B block partials of
// dotp row i (every block forms h for its slot in LDS; the block that takes the slot's
// first item also stores it, which: 0 -> hA, 1 -> hB, for the Hessenberg column).
__global__ __launch_bounds__(BLOCK) void k_axpy(const SlotDesc* D, const StepTables* T, int which) {
    __shared__ double hs[STOKES_MAX_ITERS + 1];
    const cptr<WorkList> wl = &as_const(T)->wl[WL_VEC];
    int cur = -1;
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        if (si != cur) {   // block-uniform
            __syncthreads();
            block_sum_rows(d.dotp, d.B, d.j + 1, hs);
            __syncthreads();
            if (it == wl->prefix[si]) {
                double* h = which ? d.hB : d.hA;
                for (int i = threadIdx.x; i <= d.j; i += BLOCK) h[i] = hs[i];
            }
            cur = si;
        }
        const int64_t n = 3 * (int64_t)d.N;
        const int64_t e = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (e >= n) continue;
        double acc = 0.0;
        for (int i = 0; i <= d.j; ++i) acc = fma(d.V[(int64_t)i * n + e], hs[i], acc);
        d.w[e] = d.w[e] - acc;
    }
}

// v_{j+1} = w / h_{j+1,j} with h_{j+1,j} = |w| = sqrt(the sum of the B block partials of
// w.w), 0 after a breakdown (h_{j+1,j} = 0).  The block that takes the slot's first item
// also does the Givens step on LDS copies: Hessenberg column j (hA + hB, then
// h_{j+1,j}), the previous rotations in order, the new rotation, the residual |g_{j+1}|
// and the status row.  With `arrive` (a replayed iteration), the last block to finish
// advances each listed slot's iteration counter j, once every block has read it: each
// block counts itself in after a fence, and the one that brings the count to the grid
// size resets the count and writes the counters.
__global__ __launch_bounds__(BLOCK) void k_scale_givens(SlotDesc* D, const StepTables* T, double* stat,
                                                        unsigned* arrive) {
    __shared__ double hn_s;
    __shared__ double col[STOKES_MAX_ITERS + 2], cs[STOKES_MAX_ITERS + 1], sn[STOKES_MAX_ITERS + 1];
    const cptr<WorkList> wl = &as_const(T)->wl[WL_VEC];
    int cur = -1;
    double hn = 0.0;
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        if (si != cur) {   // block-uniform
            const bool first = it == wl->prefix[si];
            const int j = d.j;
            __syncthreads();
            block_sum_rows(d.normp, d.B, 1, &hn_s);
            if (first)
                for (int i = threadIdx.x; i <= j; i += BLOCK) {
                    col[i] = d.hA[i] + d.hB[i];
                    if (i < j) {
                        cs[i] = d.cs[i];
                        sn[i] = d.sn[i];
                    }
                }
            __syncthreads();
            hn = sqrt(hn_s);
            cur = si;
            if (first) {
                if (threadIdx.x == 0) {
                    col[j + 1] = hn;
                    for (int i = 0; i < j; ++i) {
                        const double a = col[i], c = col[i + 1];
                        col[i] = cs[i] * a + sn[i] * c;
                        col[i + 1] = -sn[i] * a + cs[i] * c;
                    }
                    const double den = hypot(col[j], col[j + 1]);
                    d.cs[j] = col[j] / den;
                    d.sn[j] = col[j + 1] / den;
                    col[j] = den;
                    col[j + 1] = 0.0;
                    d.g[j + 1] = -d.sn[j] * d.g[j];
                    d.g[j] = d.cs[j] * d.g[j];
                    double* st = stat + NSTAT * d.sid;
                    st[0] = hn;
                    st[2] = fabs(d.g[j + 1]);
                    st[3] = hn == 0.0 ? 1.0 : 0.0;
                }
                __syncthreads();
                double* H = d.H + (int64_t)j * (d.k + 1);
                for (int i = threadIdx.x; i <= j + 1; i += BLOCK) H[i] = col[i];
            }
        }
        const int64_t n = 3 * (int64_t)d.N;
        const int64_t e = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (e >= n) continue;
        d.V[(int64_t)(d.j + 1) * n + e] = hn > 0.0 ? d.w[e] / hn : 0.0;
    }
    if (!arrive) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(arrive, 1u) == gridDim.x - 1) {
            for (int q = 0; q < wl->n; ++q) D[wl->slot[q]].j += 1;
            *arrive = 0u;
            __threadfence();
        }
    }
}

// ---- finalisation ----------------------------------------------------------------
// Back substitution R y = g over the m = d.j iterations done.
__global__ __launch_bounds__(BLOCK) void k_backsub(const SlotDesc* D, const StepTables* T) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_ONE];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const auto& d = as_const(D)[wl->slot[find_slot(wl, it)]];
        if (threadIdx.x != 0) continue;
        const int m = d.j;
        const int ld = d.k + 1;
        for (int i = m - 1; i >= 0; --i) {
            double s = 0.0;
            for (int l = i + 1; l < m; ++l) s += d.H[(int64_t)l * ld + i] * d.y[l];
            d.y[i] = (d.g[i] - s) / d.H[(int64_t)i * ld + i];
        }
    }
}

// w = V_m y at every node (w is free once the iterations are done).
__global__ __launch_bounds__(BLOCK) void k_vy(const SlotDesc* D, const StepTables* T) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_PRE];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int64_t i = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (i >= d.N) continue;
        const int64_t N = d.N, n = 3 * N;
        double v[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l < d.j; ++l) {
            const double yl = d.y[l];
            const double* Vl = d.V + (int64_t)l * n;
            v[0] = fma(Vl[i], yl, v[0]);
            v[1] = fma(Vl[N + i], yl, v[1]);
            v[2] = fma(Vl[2 * N + i], yl, v[2]);
        }
        d.w[i] = v[0];
        d.w[N + i] = v[1];
        d.w[2 * N + i] = v[2];
    }
}

// x = P^{-1} w at every node.
__global__ __launch_bounds__(BLOCK) void k_solution(const SlotDesc* D, const StepTables* T) {
    const cptr<WorkList> wl = &as_const(T)->wl[WL_PRE];
    for (int64_t it = blockIdx.x; it < wl->prefix[wl->n]; it += gridDim.x) {
        const int si = find_slot(wl, it);
        const auto& d = as_const(D)[wl->slot[si]];
        const int64_t i = (it - wl->prefix[si]) * BLOCK + threadIdx.x;
        if (i >= d.N) continue;
        const int64_t N = d.N;
        double x0, x1, x2;
        if (d.opts & STOKES_PRECOND_BLOCK) {
            block_apply(d.binv, i, N, d.npf, d.w, x0, x1, x2);
        } else {
            x0 = d.w[i];
            x1 = d.w[N + i];
            x2 = d.w[2 * N + i];
            apply_local(d.kappa, d.mu, true, d.tan[i], d.tan[N + i], d.tan[2 * N + i], x0, x1, x2);
        }
        d.x[i] = x0;
        d.x[N + i] = x1;
        d.x[2 * N + i] = x2;
    }
}

// ---- the nonlocal self term alone (stokes_nonlocal_sbt) --------------------------
__global__ __launch_bounds__(BLOCK) void k_fiber_tables(int64_t N, int npf, const double* flen,
                                                        double* wq, double* sarc) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= N) return;
    const int f = (int)(i / npf), kk = (int)(i % npf);
    wq[i] = cc_weight(kk, npf - 1) * 0.5 * flen[f];
    sarc[i] = 0.5 * flen[f] * (1.0 + cos(kk * 3.14159265358979323846 / (npf - 1)));
}

__global__ __launch_bounds__(BLOCK) void k_nonlocal_eval(int64_t N, int npf, const double* xyz,
                                                         const double* tan, const double* f,
                                                         const double* wq, const double* sarc,
                                                         double delta, double pref, double* out) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= N) return;
    double kx, ky, kz;
    nonlocal_at(i, N, npf, xyz, tan, f, wq, sarc, delta, pref, kx, ky, kz);
    out[i] = kx;
    out[N + i] = ky;
    out[2 * N + i] = kz;
}

// ---- host side ---------------------------------------------------------------------

// Element blocks per request for the Gram-Schmidt dot products: about one per 256
// vector elements (a thread per element and vector group), at most 256, so that
// mid-size requests also spread over many CUs.
static int32_t dot_blocks(int64_t n) {
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(256, (n + 255) / 256));
}

size_t vector_plan_bytes(int64_t n_vec, int32_t k) {
    const int64_t n = 3 * n_vec;
    const int32_t B = dot_blocks(n);
    size_t b = 0;
    auto add = [&](size_t bytes) { b += Carve::round(bytes) + 256; };
    add(n * 8);                        // rhs
    add((size_t)(k + 1) * n * 8);      // V
    add(n * 8);                        // z
    add(n * 8);                        // w
    add(n * 8);                        // x
    add((size_t)(k + 1) * B * 8);      // dotp
    add(B * 8);                        // normp
    add((k + 1) * 8);                  // hA
    add((k + 1) * 8);                  // hB
    add((size_t)(k + 1) * k * 8);      // H
    add(k * 8);                        // cs
    add(k * 8);                        // sn
    add((k + 1) * 8);                  // g
    add(k * 8);                        // y
    return b + 4096;
}

SlotPlan slot_plan(int32_t n_fib, int32_t npf, int32_t k, bool mixed, uint32_t opts) {
    SlotPlan sp{};
    const int64_t N = (int64_t)n_fib * npf;
    sp.P = make_partition(N, N, mixed ? R_SL32 : R_SL64, TARGET_BLOCKS_SLOT, MIN_TILES_PER_CHUNK);
    sp.B = dot_blocks(3 * N);
    const int64_t n = 3 * N;
    size_t b = 0;
    auto add = [&](size_t bytes) { b += Carve::round(bytes) + 256; };
    add(n * 8);               // xyz
    add(n * 8);               // tan
    add(n_fib * 8);           // flen
    add(n * 8);               // rhs
    add(N * 4);               // fib
    add(N * 8);               // wq
    add(N * 8);               // sarc
    add((opts & STOKES_PRECOND_BLOCK) ? (size_t)n_fib * 9 * npf * npf * 8 : 0);  // binv
    add((size_t)(k + 1) * n * 8);  // V
    add(n * 8);               // z
    add(n * 8);               // w
    add(n * 8);               // x
    add((size_t)(k + 1) * sp.B * 8);  // dotp
    add(sp.B * 8);            // normp
    add((k + 1) * 8);         // hA
    add((k + 1) * 8);         // hB
    add((size_t)(k + 1) * k * 8);  // H
    add(k * 8);               // cs
    add(k * 8);               // sn
    add((k + 1) * 8);         // g
    add(k * 8);               // y
    add(sp.P.n_tiles * sizeof(Tile));
    add(N * sizeof(SrcSL64));
    add(mixed ? N * sizeof(SrcSL32) : 0);
    add(mixed ? N * 4 : 0);   // near_t
    add(N * sizeof(int2));    // excl
    add((size_t)sp.P.n_chunks * n * 8);  // partial
    sp.bytes = b + 4096;
    return sp;
}

struct BatchRes {
    int dev = -1;
    SlotDesc* host_desc = nullptr;
    StepTables* host_tab = nullptr;
    double* host_stat = nullptr;
    double* lag = nullptr;   // [2][MAX_SLOTS * NSTAT]
    hipEvent_t lag_ev[2] = {nullptr, nullptr};
    SlotDesc* stage_desc[UPLOAD_RING] = {};
    StepTables* stage_tab[UPLOAD_RING] = {};
    hipEvent_t stage_ev[UPLOAD_RING] = {};
    SlotDesc* dev_desc = nullptr;
    StepTables* dev_tab = nullptr;
    double* dev_stat = nullptr;
    unsigned* dev_arrive = nullptr;   // k_scale_givens' block count (zero between launches)
    ~BatchRes() {
        for (int k = 0; k < UPLOAD_RING; ++k) {
            if (stage_ev[k]) (void)hipEventDestroy(stage_ev[k]);
            if (stage_desc[k]) (void)hipHostFree(stage_desc[k]);
            if (stage_tab[k]) (void)hipHostFree(stage_tab[k]);
        }
        for (hipEvent_t e : lag_ev)
            if (e) (void)hipEventDestroy(e);
        if (dev_desc) (void)hipFree(dev_desc);
        if (dev_tab) (void)hipFree(dev_tab);
        if (dev_stat) (void)hipFree(dev_stat);
        if (dev_arrive) (void)hipFree(dev_arrive);
        if (host_desc) (void)hipHostFree(host_desc);
        if (host_tab) (void)hipHostFree(host_tab);
        if (host_stat) (void)hipHostFree(host_stat);
        if (lag) (void)hipHostFree(lag);
    }
};

static std::mutex g_res_mu;
static std::vector<BatchRes*> g_res_free;   // kept until the process ends

static int batch_res_acquire(BatchRes** out) {
    int dev = 0;
    STOKES_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        for (size_t i = 0; i < g_res_free.size(); ++i)
            if (g_res_free[i]->dev == dev) {
                *out = g_res_free[i];
                g_res_free.erase(g_res_free.begin() + (std::ptrdiff_t)i);
                return STOKES_OK;
            }
    }
    std::unique_ptr<BatchRes> r(new BatchRes());
    r->dev = dev;
    STOKES_HIP(hipHostMalloc((void**)&r->host_desc, sizeof(SlotDesc) * MAX_SLOTS, hipHostMallocDefault));
    STOKES_HIP(hipHostMalloc((void**)&r->host_tab, sizeof(StepTables), hipHostMallocDefault));
    STOKES_HIP(hipHostMalloc((void**)&r->host_stat, sizeof(double) * NSTAT * MAX_SLOTS, hipHostMallocDefault));
    STOKES_HIP(hipHostMalloc((void**)&r->lag, 2 * sizeof(double) * NSTAT * MAX_SLOTS, hipHostMallocDefault));
    for (int k = 0; k < 2; ++k) STOKES_HIP(hipEventCreateWithFlags(&r->lag_ev[k], hipEventDisableTiming));
    for (int k = 0; k < UPLOAD_RING; ++k) {
        STOKES_HIP(hipHostMalloc((void**)&r->stage_desc[k], sizeof(SlotDesc) * MAX_SLOTS, hipHostMallocDefault));
        STOKES_HIP(hipHostMalloc((void**)&r->stage_tab[k], sizeof(StepTables), hipHostMallocDefault));
        STOKES_HIP(hipEventCreateWithFlags(&r->stage_ev[k], hipEventDisableTiming));
    }
    STOKES_HIP(hipMalloc((void**)&r->dev_desc, sizeof(SlotDesc) * MAX_SLOTS));
    STOKES_HIP(hipMalloc((void**)&r->dev_tab, sizeof(StepTables)));
    STOKES_HIP(hipMalloc((void**)&r->dev_stat, sizeof(double) * NSTAT * MAX_SLOTS));
    STOKES_HIP(hipMalloc((void**)&r->dev_arrive, sizeof(unsigned)));
    STOKES_HIP(hipMemset(r->dev_arrive, 0, sizeof(unsigned)));
    *out = r.release();
    return STOKES_OK;
}

// Back to the free list once nothing queued on the Batch's stream still reads them;
// freed instead if that wait fails.
static void batch_res_release(BatchRes* r, hipStream_t st) {
    if (!r) return;
    if (hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        delete r;
        return;
    }
    std::lock_guard<std::mutex> lk(g_res_mu);
    g_res_free.push_back(r);
}

void batch_res_drain() {
    std::vector<BatchRes*> all;
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        all.swap(g_res_free);
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (BatchRes* r : all) {
        (void)hipSetDevice(r->dev);
        delete r;
    }
    (void)hipSetDevice(cur);
}

Batch::~Batch() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    batch_res_release(res_, st_);
}

int Batch::init(hipStream_t st, bool mixed, bool doublet, bool use_graph) {
    if (res_) return fail(STOKES_E_INVAL, "Batch::init: already initialised");
    st_ = st;
    mixed_ = mixed;
    doublet_ = doublet;
    use_graph_ = use_graph;
    if (int rc = batch_res_acquire(&res_)) return rc;
    host_desc_ = res_->host_desc;
    host_tab_ = res_->host_tab;
    host_stat_ = res_->host_stat;
    dev_desc_ = res_->dev_desc;
    dev_tab_ = res_->dev_tab;
    dev_stat_ = res_->dev_stat;
    for (int k = 0; k < NSTAGE; ++k) {
        stage_[k].desc = res_->stage_desc[k];
        stage_[k].tab = res_->stage_tab[k];
        stage_[k].ev = res_->stage_ev[k];
        stage_[k].used = false;
    }
    next_stage_ = 0;
    memset(host_desc_, 0, sizeof(SlotDesc) * MAX_SLOTS);
    memset(host_tab_, 0, sizeof(StepTables));
    memset(host_stat_, 0, sizeof(double) * NSTAT * MAX_SLOTS);
    return STOKES_OK;
}

double* Batch::lag_row(int k) { return res_->lag + (size_t)(k & 1) * NSTAT * MAX_SLOTS; }
hipEvent_t Batch::lag_event(int k) { return res_->lag_ev[k & 1]; }

int Batch::attach(int s, void* mem, int32_t n_fib, int32_t npf, int32_t k, double eps, double mu,
                  double near_r, uint32_t opts, double delta, const double* xyz,
                  const double* tan, const double* flen, const double* rhs) {
    const SlotPlan sp = slot_plan(n_fib, npf, k, mixed_, opts);
    const int64_t N = (int64_t)n_fib * npf, n = 3 * N;
    Carve c(mem);
    SlotDesc d{};
    d.N = (int32_t)N;
    d.n_fib = n_fib;
    d.npf = npf;
    d.k = k;
    d.j = 0;
    d.B = sp.B;
    d.n_items_vec = (int32_t)((n + BLOCK - 1) / BLOCK);
    d.n_items_node = (int32_t)((N + BLOCK - 1) / BLOCK);
    d.n_items_sl = sp.P.n_tblocks * ((opts & OPT_FAR) ? 1 : sp.P.n_chunks);   // far: k_red sums one row
    d.sid = s;
    d.opts = opts & (STOKES_NONLOCAL | STOKES_PRECOND_BLOCK | OPT_FAR);
    d.delta = delta;
    d.eps = eps;
    d.mu = mu;
    d.kappa = -log(eps * eps * M_E);
    d.pref = 1.0 / (8.0 * 3.14159265358979323846 * mu);
    d.near_r = mixed_ ? std::max(near_r, 0.0) : 0.0;
    double* xyz_d = c.take<double>(n);
    double* tan_d = c.take<double>(n);
    double* flen_d = c.take<double>(n_fib);
    double* rhs_d = c.take<double>(n);
    d.xyz = xyz_d;
    d.tan = tan_d;
    d.flen = flen_d;
    d.rhs = rhs_d;
    d.fib = c.take<int32_t>(N);
    d.wq = c.take<double>(N);
    d.sarc = c.take<double>(N);
    d.binv = (opts & STOKES_PRECOND_BLOCK) ? c.take<double>((size_t)n_fib * 9 * npf * npf) : nullptr;
    d.V = c.take<double>((size_t)(k + 1) * n);
    d.z = c.take<double>(n);
    d.w = c.take<double>(n);
    d.x = c.take<double>(n);
    d.dotp = c.take<double>((size_t)(k + 1) * sp.B);
    d.normp = c.take<double>(sp.B);
    d.hA = c.take<double>(k + 1);
    d.hB = c.take<double>(k + 1);
    d.H = c.take<double>((size_t)(k + 1) * k);
    d.cs = c.take<double>(k);
    d.sn = c.take<double>(k);
    d.g = c.take<double>(k + 1);
    d.y = c.take<double>(k);
    d.tiles = c.take<Tile>(sp.P.n_tiles);
    d.s64 = c.take<SrcSL64>(N);
    d.s32 = c.take<SrcSL32>(mixed_ ? N : 0);
    d.near_t = c.take<float>(mixed_ ? N : 0);
    d.excl = c.take<int2>(N);
    d.partial = c.take<double>((size_t)sp.P.n_chunks * n);
    if (c.off > sp.bytes) return fail(STOKES_E_INVAL, "slot layout exceeds its plan");
    if (!mixed_) {
        d.s32 = nullptr;
        d.near_t = nullptr;
    }
    SumArgs& a = d.sl;
    a.tx = xyz_d;
    a.t_stride = N;
    a.n_t = N;
    a.excl = d.excl;
    a.tiles = d.tiles;
    a.n_tiles = sp.P.n_tiles;
    a.tiles_per_chunk = sp.P.tiles_per_chunk;
    a.n_tblocks = sp.P.n_tblocks;
    a.s64 = d.s64;
    a.s32 = d.s32;
    a.near_t = d.near_t;
    a.n_s = N;
    a.partial = d.partial;
    a.counters = nullptr;
    STOKES_HIP(hipMemcpyAsync(xyz_d, xyz, n * 8, hipMemcpyDefault, st_));
    STOKES_HIP(hipMemcpyAsync(tan_d, tan, n * 8, hipMemcpyDefault, st_));
    STOKES_HIP(hipMemcpyAsync(flen_d, flen, (size_t)n_fib * 8, hipMemcpyDefault, st_));
    STOKES_HIP(hipMemcpyAsync(rhs_d, rhs, n * 8, hipMemcpyDefault, st_));
    host_desc_[s] = d;
    return STOKES_OK;
}

void Batch::set_list(WL w, const std::vector<int>& slots) {
    WorkList& L = host_tab_->wl[w];
    L.n = (int32_t)slots.size();
    L.prefix[0] = 0;
    for (size_t q = 0; q < slots.size(); ++q) {
        const SlotDesc& d = host_desc_[slots[q]];
        int64_t items = 0;
        switch (w) {
            case WL_PRE: items = d.n_items_node; break;   // >= tiles / BLOCK as well
            case WL_SL: items = d.n_items_sl; break;
            case WL_RED: items = d.n_items_node; break;
            case WL_DOT: items = (int64_t)d.B * dot_groups(d.k); break;
            case WL_ONE: items = 1; break;
            case WL_VEC: items = d.n_items_vec; break;
            case WL_FIB: items = (d.opts & STOKES_PRECOND_BLOCK) ? d.n_fib : 0; break;
            default: break;
        }
        L.slot[q] = slots[q];
        L.base[q] = 0;
        L.prefix[q + 1] = L.prefix[q] + items;
    }
}

void Batch::set_sl_list(const std::vector<Part>& parts) {
    WorkList& L = host_tab_->wl[WL_SL];
    L.n = 0;
    L.prefix[0] = 0;
    for (const Part& p : parts) {
        if (p.sl_count <= 0) continue;
        L.slot[L.n] = p.slot;
        L.base[L.n] = p.sl_begin;
        L.prefix[L.n + 1] = L.prefix[L.n] + p.sl_count;
        ++L.n;
    }
}

int Batch::upload() {
    Stage& g = stage_[next_stage_];
    next_stage_ = (next_stage_ + 1) % NSTAGE;
    if (g.used) STOKES_HIP(hipEventSynchronize(g.ev));   // its last copy has been read
    memcpy(g.desc, host_desc_, sizeof(SlotDesc) * MAX_SLOTS);
    memcpy(g.tab, host_tab_, sizeof(StepTables));
    STOKES_HIP(hipMemcpyAsync(dev_desc_, g.desc, sizeof(SlotDesc) * MAX_SLOTS, hipMemcpyHostToDevice, st_));
    STOKES_HIP(hipMemcpyAsync(dev_tab_, g.tab, sizeof(StepTables), hipMemcpyHostToDevice, st_));
    STOKES_HIP(hipEventRecord(g.ev, st_));
    g.used = true;
    return STOKES_OK;
}

static unsigned grid_for(const WorkList& L, int cap) {
    const int64_t t = L.prefix[L.n];
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(t, cap));
}

int Batch::copy_status_async(double* dst, hipStream_t s) {
    STOKES_HIP(hipMemcpyAsync(dst, dev_stat_, sizeof(double) * NSTAT * MAX_SLOTS, hipMemcpyDeviceToHost,
                              s ? s : st_));
    return STOKES_OK;
}
int Batch::read_status() {
    STOKES_HIP(hipMemcpyAsync(host_stat_, dev_stat_, sizeof(double) * NSTAT * MAX_SLOTS,
                              hipMemcpyDeviceToHost, st_));
    STOKES_HIP(hipStreamSynchronize(st_));
    return STOKES_OK;
}

int Batch::start(const std::vector<int>& slots) {
    if (slots.empty()) return STOKES_OK;
    set_list(WL_PRE, slots);
    set_list(WL_DOT, slots);
    set_list(WL_ONE, slots);
    set_list(WL_VEC, slots);
    set_list(WL_FIB, slots);
    int rc = upload();
    if (rc) return rc;
    const StepTables& T = *host_tab_;
    hipLaunchKernelGGL(k_geom, dim3(grid_for(T.wl[WL_PRE], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    hipLaunchKernelGGL(k_tiles, dim3(grid_for(T.wl[WL_PRE], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    if (T.wl[WL_FIB].prefix[T.wl[WL_FIB].n] > 0)
        hipLaunchKernelGGL(k_block, dim3(grid_for(T.wl[WL_FIB], 4096)), dim3(BLOCK_GJ), 0, st_, dev_desc_, dev_tab_);
    hipLaunchKernelGGL(k_init_norm, dim3(grid_for(T.wl[WL_DOT], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    hipLaunchKernelGGL(k_init_beta, dim3(grid_for(T.wl[WL_ONE], G_ONE)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_, dev_stat_);
    hipLaunchKernelGGL(k_init_v0, dim3(grid_for(T.wl[WL_VEC], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    STOKES_HIP(hipGetLastError());
    return read_status();
}

int Batch::launch_step(bool graph_sizes) {
    const StepTables& T = *host_tab_;
    auto g = [&](WL w, int cap) { return graph_sizes ? (unsigned)cap : grid_for(T.wl[w], cap); };
    const dim3 b(BLOCK);
    hipLaunchKernelGGL(k_pre, dim3(g(WL_PRE, G_ELEM)), b, 0, st_, dev_desc_, dev_tab_, doublet_ ? 1 : 0);
    if (!graph_sizes) prof_begin(st_);   // (events are not recorded into a captured graph)
    if (mixed_) {
        if (doublet_) hipLaunchKernelGGL((k_sl<true, true>), dim3(g(WL_SL, G_SL)), b, 0, st_, dev_desc_, dev_tab_);
        else hipLaunchKernelGGL((k_sl<true, false>), dim3(g(WL_SL, G_SL)), b, 0, st_, dev_desc_, dev_tab_);
    } else {
        if (doublet_) hipLaunchKernelGGL((k_sl<false, true>), dim3(g(WL_SL, G_SL)), b, 0, st_, dev_desc_, dev_tab_);
        else hipLaunchKernelGGL((k_sl<false, false>), dim3(g(WL_SL, G_SL)), b, 0, st_, dev_desc_, dev_tab_);
    }
    if (!graph_sizes) prof_end(st_);
    hipLaunchKernelGGL(k_red, dim3(g(WL_RED, G_ELEM)), b, 0, st_, dev_desc_, dev_tab_);
    return launch_ortho(graph_sizes);
}

int Batch::launch_ortho(bool graph_sizes, bool advance) {
    const StepTables& T = *host_tab_;
    auto g = [&](WL w, int cap) { return graph_sizes ? (unsigned)cap : grid_for(T.wl[w], cap); };
    const dim3 b(BLOCK);
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_dot, dim3(g(WL_DOT, G_ELEM)), b, 0, st_, dev_desc_, dev_tab_, pass);
        hipLaunchKernelGGL(k_axpy, dim3(g(WL_VEC, G_ELEM)), b, 0, st_, dev_desc_, dev_tab_, pass);
    }
    hipLaunchKernelGGL(k_dot, dim3(g(WL_DOT, G_ELEM)), b, 0, st_, dev_desc_, dev_tab_, 2);
    hipLaunchKernelGGL(k_scale_givens, dim3(g(WL_VEC, G_ELEM)), b, 0, st_, dev_desc_, dev_tab_, dev_stat_,
                       advance ? res_->dev_arrive : (unsigned*)nullptr);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

int Batch::launch_pre(const std::vector<int>& slots) {
    set_list(WL_PRE, slots);
    if (int rc = upload()) return rc;
    hipLaunchKernelGGL(k_pre, dim3(grid_for(host_tab_->wl[WL_PRE], G_ELEM)), dim3(BLOCK), 0, st_, dev_desc_,
                       dev_tab_, doublet_ ? 1 : 0);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

int Batch::launch_red_ortho(const std::vector<int>& slots) {
    set_list(WL_RED, slots);
    set_list(WL_DOT, slots);
    set_list(WL_ONE, slots);
    set_list(WL_VEC, slots);
    if (int rc = upload()) return rc;
    hipLaunchKernelGGL(k_red, dim3(grid_for(host_tab_->wl[WL_RED], G_ELEM)), dim3(BLOCK), 0, st_, dev_desc_,
                       dev_tab_);
    return launch_ortho(false);
}

int Batch::step(const std::vector<int>& slots) {
    if (slots.empty()) return STOKES_OK;
    set_list(WL_PRE, slots);
    set_list(WL_SL, slots);
    set_list(WL_RED, slots);
    set_list(WL_DOT, slots);
    set_list(WL_ONE, slots);
    set_list(WL_VEC, slots);
    return run_step();
}

int Batch::set_step_lists(const std::vector<Part>& parts) {
    std::vector<int> begin, end;
    for (const Part& p : parts) {
        const int32_t n = host_desc_[p.slot].n_items_sl;
        if (p.sl_begin < 0 || p.sl_count < 0 || p.sl_begin + p.sl_count > n)
            return fail(STOKES_E_INVAL, "step_parts: single-layer item range out of bounds");
        if (p.sl_begin == 0) begin.push_back(p.slot);
        if (p.sl_begin + p.sl_count == n) end.push_back(p.slot);
    }
    set_list(WL_PRE, begin);
    set_sl_list(parts);
    set_list(WL_RED, end);
    set_list(WL_DOT, end);
    set_list(WL_ONE, end);
    set_list(WL_VEC, end);
    return STOKES_OK;
}

int Batch::step_parts(const std::vector<Part>& parts) {
    if (parts.empty()) return STOKES_OK;
    if (int rc = set_step_lists(parts)) return rc;
    return run_step();
}

int Batch::step_parts_nowait(const std::vector<Part>& parts) {
    if (parts.empty()) return STOKES_OK;
    if (int rc = set_step_lists(parts)) return rc;
    return launch_or_replay();
}

int Batch::run_step() {
    if (int rc = launch_or_replay()) return rc;
    return read_status();
}

int Batch::launch_or_replay() {
    int rc = upload();
    if (rc) return rc;
    if (use_graph_) {
        if (!exec_) {
            STOKES_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
            rc = launch_step(true);
            hipGraph_t gr = nullptr;
            hipError_t e = hipStreamEndCapture(st_, &gr);
            if (rc) {
                if (gr) (void)hipGraphDestroy(gr);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            graph_ = gr;
            STOKES_HIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
        }
        STOKES_HIP(hipGraphLaunch(exec_, st_));
    } else {
        if ((rc = launch_step(false))) return rc;
    }
    return STOKES_OK;
}

int Batch::finalize(const std::vector<int>& slots) {
    if (slots.empty()) return STOKES_OK;
    set_list(WL_PRE, slots);
    set_list(WL_ONE, slots);
    int rc = upload();
    if (rc) return rc;
    const StepTables& T = *host_tab_;
    hipLaunchKernelGGL(k_backsub, dim3(grid_for(T.wl[WL_ONE], G_ONE)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    hipLaunchKernelGGL(k_vy, dim3(grid_for(T.wl[WL_PRE], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    hipLaunchKernelGGL(k_solution, dim3(grid_for(T.wl[WL_PRE], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

int Batch::attach_vector(int s, void* mem, int64_t n_vec, int32_t k, const double* rhs) {
    const int64_t n = 3 * n_vec;
    Carve c(mem);
    SlotDesc d{};
    d.N = (int32_t)n_vec;
    d.k = k;
    d.j = 0;
    d.B = dot_blocks(n);
    d.n_items_vec = (int32_t)((n + BLOCK - 1) / BLOCK);
    d.n_items_node = (int32_t)((n_vec + BLOCK - 1) / BLOCK);
    d.n_items_sl = 0;
    d.sid = s;
    double* rhs_d = c.take<double>(n);
    d.rhs = rhs_d;
    d.V = c.take<double>((size_t)(k + 1) * n);
    d.z = c.take<double>(n);
    d.w = c.take<double>(n);
    d.x = c.take<double>(n);
    d.dotp = c.take<double>((size_t)(k + 1) * d.B);
    d.normp = c.take<double>(d.B);
    d.hA = c.take<double>(k + 1);
    d.hB = c.take<double>(k + 1);
    d.H = c.take<double>((size_t)(k + 1) * k);
    d.cs = c.take<double>(k);
    d.sn = c.take<double>(k);
    d.g = c.take<double>(k + 1);
    d.y = c.take<double>(k);
    if (c.off > vector_plan_bytes(n_vec, k)) return fail(STOKES_E_INVAL, "vector slot layout exceeds its plan");
    STOKES_HIP(hipMemcpyAsync(rhs_d, rhs, n * 8, hipMemcpyDeviceToDevice, st_));
    host_desc_[s] = d;
    return STOKES_OK;
}

int Batch::start_vector(const std::vector<int>& slots) {
    if (slots.empty()) return STOKES_OK;
    set_list(WL_PRE, {});
    set_list(WL_SL, {});
    set_list(WL_RED, {});
    set_list(WL_FIB, {});
    set_list(WL_DOT, slots);
    set_list(WL_ONE, slots);
    set_list(WL_VEC, slots);
    int rc = upload();
    if (rc) return rc;
    const StepTables& T = *host_tab_;
    hipLaunchKernelGGL(k_init_norm, dim3(grid_for(T.wl[WL_DOT], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    hipLaunchKernelGGL(k_init_beta, dim3(grid_for(T.wl[WL_ONE], G_ONE)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_, dev_stat_);
    hipLaunchKernelGGL(k_init_v0, dim3(grid_for(T.wl[WL_VEC], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    STOKES_HIP(hipGetLastError());
    return read_status();
}

int Batch::step_ortho(const std::vector<int>& slots) {
    if (slots.empty()) return STOKES_OK;
    if (int rc = step_ortho_nowait(slots)) return rc;
    return read_status();
}

int Batch::step_ortho_nowait(const std::vector<int>& slots) {
    if (slots.empty()) return STOKES_OK;
    set_list(WL_DOT, slots);
    set_list(WL_ONE, slots);
    set_list(WL_VEC, slots);
    int rc = upload();
    if (rc) return rc;
    return launch_ortho(false);
}

int Batch::ortho_lists(const std::vector<int>& slots) {
    set_list(WL_DOT, slots);
    set_list(WL_ONE, slots);
    set_list(WL_VEC, slots);
    return upload();
}

int Batch::launch_ortho_fixed(const std::vector<int>& slots, hipStream_t s) {
    if (slots.empty()) return STOKES_OK;
    const hipStream_t own = st_;
    st_ = s;
    const int rc = launch_ortho(false, true);
    st_ = own;
    return rc;
}

int Batch::finalize_vector(const std::vector<int>& slots) {
    if (slots.empty()) return STOKES_OK;
    set_list(WL_PRE, slots);
    set_list(WL_ONE, slots);
    int rc = upload();
    if (rc) return rc;
    const StepTables& T = *host_tab_;
    hipLaunchKernelGGL(k_backsub, dim3(grid_for(T.wl[WL_ONE], G_ONE)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    hipLaunchKernelGGL(k_vy, dim3(grid_for(T.wl[WL_PRE], 4096)), dim3(BLOCK), 0, st_, dev_desc_, dev_tab_);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

}  // namespace stokes

using namespace stokes;

extern "C" int stokes_nonlocal_sbt(int32_t n_fib, int32_t nodes_per_fib, const double* xyz,
                                   const double* tangent, const double* fiber_len, const double* f,
                                   double delta, double mu, double* out, void* stream) {
    if (n_fib < 0 || nodes_per_fib < 2 || nodes_per_fib > 64)
        return fail(STOKES_E_INVAL, "stokes_nonlocal_sbt: need n_fib >= 0 and 2 <= nodes_per_fib <= 64");
    if (!(mu > 0.0)) return fail(STOKES_E_INVAL, "stokes_nonlocal_sbt: mu must be > 0");
    if (!(delta > 0.0) || !std::isfinite(delta))
        return fail(STOKES_E_INVAL, "stokes_nonlocal_sbt: delta must be finite and > 0");
    const int64_t N = (int64_t)n_fib * nodes_per_fib;
    if (N >= (int64_t)1 << 30) return fail(STOKES_E_INVAL, "stokes_nonlocal_sbt: too many nodes");
    if (N == 0) return STOKES_OK;
    if (!xyz || !tangent || !fiber_len || !f || !out)
        return fail(STOKES_E_INVAL, "stokes_nonlocal_sbt: null pointer");
    if (out == f) return fail(STOKES_E_INVAL, "stokes_nonlocal_sbt: out must not alias f");
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace* ws = nullptr;
    int rc = workspace_get(st, (size_t)(2 * N) * sizeof(double), &ws);
    if (rc) return rc;
    double* wq = static_cast<double*>(ws->dev);
    double* sarc = wq + N;
    const unsigned grid = (unsigned)((N + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL(k_fiber_tables, dim3(grid), dim3(BLOCK), 0, st, N, nodes_per_fib, fiber_len,
                       wq, sarc);
    hipLaunchKernelGGL(k_nonlocal_eval, dim3(grid), dim3(BLOCK), 0, st, N, nodes_per_fib, xyz,
                       tangent, f, wq, sarc, delta, 1.0 / (8.0 * 3.14159265358979323846 * mu), out);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

extern "C" int stokes_mobility_solve(int32_t n_fib, int32_t nodes_per_fib, const double* xyz,
                                     const double* tangent, const double* fiber_len,
                                     const double* rhs, double eps, double mu, double delta,
                                     int32_t iters, uint32_t flags, double* f_out,
                                     double* resid_out, int32_t* iters_out, const stokes_far* far,
                                     void* stream) {
    if (flags & ~(STOKES_PREC_MIXED | STOKES_NO_DOUBLET | STOKES_NONLOCAL | STOKES_PRECOND_BLOCK))
        return fail(STOKES_E_INVAL, "stokes_mobility_solve: unknown flag bits");
    if (int rc = check_far(far, "stokes_mobility_solve")) return rc;
    if ((flags & STOKES_NONLOCAL) && (!(delta > 0.0) || !std::isfinite(delta)))
        return fail(STOKES_E_INVAL, "stokes_mobility_solve: delta must be finite and > 0 with STOKES_NONLOCAL");
    if (n_fib < 0 || nodes_per_fib < 2 || nodes_per_fib > 64)
        return fail(STOKES_E_INVAL, "stokes_mobility_solve: need n_fib >= 0 and 2 <= nodes_per_fib <= 64");
    if (iters < 1 || iters > STOKES_MAX_ITERS)
        return fail(STOKES_E_INVAL, "stokes_mobility_solve: iters out of range");
    if (!(mu > 0.0)) return fail(STOKES_E_INVAL, "stokes_mobility_solve: mu must be > 0");
    if (!(eps > 0.0 && eps < 0.5)) return fail(STOKES_E_INVAL, "stokes_mobility_solve: eps must be in (0, 0.5)");
    const int64_t N = (int64_t)n_fib * nodes_per_fib;
    if (N >= (int64_t)1 << 30) return fail(STOKES_E_INVAL, "stokes_mobility_solve: too many nodes");
    if (N > 0 && (!xyz || !tangent || !fiber_len || !rhs || !f_out))
        return fail(STOKES_E_INVAL, "stokes_mobility_solve: null pointer");
    if (N == 0) {
        if (resid_out) *resid_out = 0.0;
        if (iters_out) *iters_out = 0;
        return STOKES_OK;
    }
    Range range("stokes_mobility_solve");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool mixed = flags & STOKES_PREC_MIXED;
    const uint32_t opts = flags & (STOKES_NONLOCAL | STOKES_PRECOND_BLOCK);
    const SlotPlan sp = slot_plan(n_fib, nodes_per_fib, iters, mixed, opts);
    Workspace* ws = nullptr;
    int rc = workspace_get(st, sp.bytes, &ws);
    if (rc) return rc;
    FarPlan fp;
    if (far && (rc = fp.make(N, xyz, *far, st))) return rc;
    Batch b;
    if ((rc = b.init(st, mixed, !(flags & STOKES_NO_DOUBLET), false))) return rc;
    if ((rc = b.attach(0, ws->dev, n_fib, nodes_per_fib, iters, eps, mu, 0.0, far ? opts | OPT_FAR : opts, delta,
                       xyz, tangent, fiber_len, rhs)))
        return rc;
    std::vector<int> one{0};
    if ((rc = b.start(one))) return rc;
    // the treecode's u_bar: Clenshaw-Curtis weights x L/2 and the fiber ids of the slot
    const uint32_t tflags = (flags & (STOKES_PREC_MIXED | STOKES_NO_DOUBLET)) | STOKES_EXCL_SAME_FIBER;
    auto far_sum = [&](int q) {
        const SlotDesc& d = b.desc(q);
        return stokes_tree_sl_eval(fp.t, d.z, d.wq, d.fib, d.n_fib, d.flen, mu, eps, 0.0, tflags, d.partial, st);
    };
    int done = 0;
    double resid = b.status(0)[2];
    if (b.status(0)[3] == 0.0) {
        for (int j = 0; j < iters; ++j) {
            b.desc(0).j = j;
            if ((rc = far ? b.step_external(one, far_sum) : b.step(one))) return rc;
            done = j + 1;
            resid = b.status(0)[2];
            if (b.status(0)[3] != 0.0) break;   // exact breakdown
        }
    }
    b.desc(0).j = done;
    if ((rc = b.finalize(one))) return rc;
    STOKES_HIP(hipMemcpyAsync(f_out, b.desc(0).x, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, st));
    STOKES_HIP(hipStreamSynchronize(st));
    if (resid_out) *resid_out = resid;
    if (iters_out) *iters_out = done;
    return STOKES_OK;
}
