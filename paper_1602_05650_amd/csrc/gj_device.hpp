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
__device__ __forceinline__ void gj_invert(int m, bool act, int r, int g, double (&A)[GJ_COLS], GjLds& s,
                                          double* X) {
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
            if (c < m) X[(int64_t)s.perm[c] * m + r] = A[jj];
        }
    }
}

}  // namespace stokes
