// Gauss-Jordan inversion with partial pivoting of one m x m matrix (m <= GJ_MAX)
// held in the registers of a workgroup of BLOCK_GJ threads: thread t owns row
// r = t % m and the columns c = g + GJ_G jj (g = t / m, jj < GJ_COLS) when
// t < GJ_G m, so every pivot step only exchanges the pivot column and row
// through LDS.  Used for the fiber self blocks of the block-Jacobi preconditioners.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stokes {

constexpr int BLOCK_GJ = 1024;
constexpr int GJ_MAX = 192;
constexpr int GJ_G = 5;                                 // column groups: GJ_G * GJ_MAX <= BLOCK_GJ
constexpr int GJ_COLS = (GJ_MAX + GJ_G - 1) / GJ_G;     // columns per thread

struct GjLds {
    double col[GJ_MAX], row[GJ_MAX], swap[2][GJ_MAX], wv[BLOCK_GJ / 64];
    int wi[BLOCK_GJ / 64], perm[GJ_MAX], dest[GJ_MAX];
};

// A holds this thread's entries A[r][g + GJ_G jj] on entry (zero where the thread is
// inactive or the column is >= m).  On return X (column-major, m x m) holds the
// inverse.  A column without a finite pivot leaves the pivot in place (the result
// is then not finite).  Every thread of the workgroup must call it.
// (act, r, g) are the thread's role as set out above: act = t < GJ_G m, r = t % m,
// g = t / m (both 0 when inactive).
// ds (LDS or null): the result's column j is multiplied by ds[j] (the inverse of a
// row-equilibrated matrix D B gives B^-1 = (D B)^-1 D).
__device__ __forceinline__ void gj_invert(int m, bool act, int r, int g, double (&A)[GJ_COLS], GjLds& s,
                                          double* X, const double* ds = nullptr) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int p = 0; p < m; ++p) {
        const int gp = p % GJ_G, jp = p / GJ_G;
        // pivot: largest |A[r][p]| over rows r >= p (smallest r on ties)
        double bv = -1.0;
        int bi = m;
        if (act && g == gp) {
            double v = 0.0;
#pragma unroll
            for (int jj = 0; jj < GJ_COLS; ++jj)
                if (jj == jp) v = A[jj];
            if (r >= p) {
                bv = fabs(v);
                bi = r;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            s.wv[wave] = bv;
            s.wi[wave] = bi;
        }
        __syncthreads();
        double pv = s.wv[0];
        int pr = s.wi[0];
        for (int w = 1; w < BLOCK_GJ / 64; ++w)
            if (s.wv[w] > pv || (s.wv[w] == pv && s.wi[w] < pr)) {
                pv = s.wv[w];
                pr = s.wi[w];
            }
        if (pr >= m) pr = p;    // (a column of NaN: no row qualifies)
        if (t == 0) s.perm[p] = pr;
        // row interchange p <-> pr through LDS
        if (pr != p) {
            if (act && (r == p || r == pr)) {
#pragma unroll
                for (int jj = 0; jj < GJ_COLS; ++jj) {
                    const int c = g + GJ_G * jj;
                    if (c < m) s.swap[r == p ? 0 : 1][c] = A[jj];
                }
            }
            __syncthreads();
            if (act && (r == p || r == pr)) {
#pragma unroll
                for (int jj = 0; jj < GJ_COLS; ++jj) {
                    const int c = g + GJ_G * jj;
                    if (c < m) A[jj] = s.swap[r == p ? 1 : 0][c];
                }
            }
        }
        // pivot column and (unscaled) pivot row to LDS
        if (act && g == gp) {
            double v = 0.0;
#pragma unroll
            for (int jj = 0; jj < GJ_COLS; ++jj)
                if (jj == jp) v = A[jj];
            s.col[r] = v;
        }
        if (act && r == p) {
#pragma unroll
            for (int jj = 0; jj < GJ_COLS; ++jj) {
                const int c = g + GJ_G * jj;
                if (c < m) s.row[c] = A[jj];
            }
        }
        __syncthreads();
        const double inv = 1.0 / s.col[p];
        const double cr = s.col[r];
        if (act) {
#pragma unroll
            for (int jj = 0; jj < GJ_COLS; ++jj) {
                const int c = g + GJ_G * jj;
                if (c < m) {
                    const double rp = c == p ? inv : s.row[c] * inv;
                    A[jj] = r == p ? rp : (c == p ? 0.0 : A[jj]) - cr * rp;
                }
            }
        }
        __syncthreads();
    }
    // undo the row interchanges on the columns (last first): column c of the
    // inverse is working column s.dest^{-1}(c)
    if (t == 0) {
        for (int c = 0; c < m; ++c) s.dest[c] = c;   // s.dest[c]: working column at c
        for (int p = m - 1; p >= 0; --p) {
            const int q = s.perm[p];
            const int a = s.dest[p];
            s.dest[p] = s.dest[q];
            s.dest[q] = a;
        }
        for (int c = 0; c < m; ++c) s.perm[s.dest[c]] = c;       // working column -> final column
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int jj = 0; jj < GJ_COLS; ++jj) {
            const int c = g + GJ_G * jj;
            if (c < m) X[(int64_t)s.perm[c] * m + r] = ds ? A[jj] * ds[s.perm[c]] : A[jj];
        }
    }
}

}  // namespace stokes

namespace stokes {

// A second layout for blocks of m <= 128 with 256 threads: thread t owns row r = t % m
// and the contiguous columns g * 64 + jj (g = t / m < 2, jj < 64) when t < 2 m.  A wave
// then holds one column range for 64 rows, so the pivot row is read from LDS as a
// broadcast and the pivot column sits at the same register index in the whole wave.
constexpr int GJ64_T = 256;
constexpr int GJ64_MAX = 128;

struct Gj64Lds {
    double col[2][GJ64_MAX], row[2][GJ64_MAX], oh[2][GJ64_MAX], kv[2][GJ64_MAX];
    unsigned wk[2][GJ64_T / 64];
    int perm[GJ64_MAX], dest[GJ64_MAX];
};

// Same contract as gj_invert: A holds A[r][g * 64 + jj] (zero beyond m); on return X
// (column-major, m x m) holds the inverse.  Every thread of the workgroup must call it.
// Partial pivoting without row interchanges: the pivot of column p is the largest
// |a_rp| over rows not yet used (to a relative 2^-13: the search compares the high
// 32 bits of |a_rp|), pi(p) records it, and the stored result S gives
// A^-1[pi^-1(a)][pi(b)] = S[a][b].  The pivot loop has no branches on the column
// index: rows are padded with zeros to 128 columns, the pivot column is a one-hot
// vector oh in LDS, a thread's entry in column p is sum_jj A[jj] oh[c], and the update
// is A <- A kv[c] - (a_rp / a_pp) row[c] with kv = 1 - oh and row carrying 1 at column p
// (the pivot row starts from 0 with a_rp = -1).  The LDS vectors alternate between two
// buffers by the parity of p, so one pivot step needs two barriers.
// ds as for gj_invert.
__device__ __forceinline__ void gj_invert64(int m, bool act, int r, int g, double (&A)[64], Gj64Lds& s,
                                            double* X, const double* ds = nullptr) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t < GJ64_MAX) {
        s.oh[0][t] = t == 0 ? 1.0 : 0.0;
        s.oh[1][t] = 0.0;
        s.kv[0][t] = t == 0 ? 0.0 : 1.0;
        s.kv[1][t] = 1.0;
    }
    bool used = false;
    __syncthreads();
    for (int p = 0; p < m; ++p) {
        const int gp = p >> 6, b = p & 1;
        const double* oh = s.oh[b];
        double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;   // this thread's entry of column p
#pragma unroll
        for (int jj = 0; jj < 64; jj += 4) {
            q0 = fma(A[jj], oh[g * 64 + jj], q0);
            q1 = fma(A[jj + 1], oh[g * 64 + jj + 1], q1);
            q2 = fma(A[jj + 2], oh[g * 64 + jj + 2], q2);
            q3 = fma(A[jj + 3], oh[g * 64 + jj + 3], q3);
        }
        const double pc = (q0 + q1) + (q2 + q3);          // (one term is nonzero)
        // pivot search key: the high word of |a_rp| with its low 7 bits replaced by
        // 127 - r (largest |a| to 2^-13, then smallest row); 0 for used rows
        unsigned key = 0u;
        if (act && g == gp) {
            s.col[b][r] = pc;
            if (!used)
                key = ((unsigned)(__double_as_longlong(fabs(pc)) >> 32) & 0xFFFFFF80u) | (unsigned)(127 - r);
        }
        for (int o = 32; o > 0; o >>= 1) key = max(key, (unsigned)__shfl_xor((int)key, o));
        if (lane == 0) s.wk[b][wave] = key;
        __syncthreads();
        unsigned kb = s.wk[b][0];
        for (int w = 1; w < GJ64_T / 64; ++w) kb = max(kb, s.wk[b][w]);
        const int pr = 127 - (int)(kb & 0x7Fu);
        if (t == 0) {
            s.perm[p] = pr;
            double* on = s.oh[b ^ 1];       // next pivot's one-hot (last read at p - 1)
            double* kn = s.kv[b ^ 1];
            if (p >= 1) {
                on[p - 1] = 0.0;
                kn[p - 1] = 1.0;
            }
            if (p + 1 < m) {
                on[p + 1] = 1.0;
                kn[p + 1] = 0.0;
            }
        }
        const bool piv = act && r == pr;
        if (piv) {          // publish the pivot row (1 at column p), then start it from 0
#pragma unroll
            for (int jj = 0; jj < 64; ++jj) {
                const double o = oh[g * 64 + jj];
                s.row[b][g * 64 + jj] = fma(A[jj], 1.0 - o, o);
                A[jj] = 0.0;
            }
            used = true;
        }
        __syncthreads();
        const double inv = 1.0 / s.col[b][pr];
        const double crinv = (piv ? -1.0 : s.col[b][r]) * inv;
        const double* kv = s.kv[b];
        if (act) {
#pragma unroll
            for (int jj = 0; jj < 64; ++jj) {
                const int c = g * 64 + jj;
                A[jj] = fma(A[jj], kv[c], -crinv * s.row[b][c]);
            }
        }
    }
    __syncthreads();
    if (t == 0)
        for (int p = 0; p < m; ++p) s.dest[s.perm[p]] = p;     // pi^-1
    __syncthreads();
    if (act) {
        const int row_out = s.dest[r];
#pragma unroll
        for (int jj = 0; jj < 64; ++jj) {
            const int c = g * 64 + jj;
            if (c < m) X[(int64_t)s.perm[c] * m + row_out] = ds ? A[jj] * ds[s.perm[c]] : A[jj];
        }
    }
}

}  // namespace stokes
