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
    double col[2][GJ64_MAX], row[2][GJ64_MAX], inv[2];
    unsigned wk[2][GJ64_T / 64];
    int perm[GJ64_MAX], dest[GJ64_MAX];
};

// Register j of A for an index j uniform over the wave: a switch on j (scalar
// branches) around one register move per case.  The moves are written as inline asm
// so that the cases cannot be folded into an indexed access, which would move A to
// scratch memory.
__device__ __forceinline__ double reg_get64(const double (&A)[64], int j) {
    double v = 0.0;
    switch (j) {
    case 0: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[0])); break;
    case 1: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[1])); break;
    case 2: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[2])); break;
    case 3: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[3])); break;
    case 4: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[4])); break;
    case 5: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[5])); break;
    case 6: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[6])); break;
    case 7: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[7])); break;
    case 8: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[8])); break;
    case 9: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[9])); break;
    case 10: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[10])); break;
    case 11: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[11])); break;
    case 12: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[12])); break;
    case 13: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[13])); break;
    case 14: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[14])); break;
    case 15: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[15])); break;
    case 16: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[16])); break;
    case 17: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[17])); break;
    case 18: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[18])); break;
    case 19: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[19])); break;
    case 20: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[20])); break;
    case 21: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[21])); break;
    case 22: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[22])); break;
    case 23: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[23])); break;
    case 24: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[24])); break;
    case 25: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[25])); break;
    case 26: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[26])); break;
    case 27: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[27])); break;
    case 28: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[28])); break;
    case 29: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[29])); break;
    case 30: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[30])); break;
    case 31: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[31])); break;
    case 32: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[32])); break;
    case 33: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[33])); break;
    case 34: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[34])); break;
    case 35: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[35])); break;
    case 36: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[36])); break;
    case 37: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[37])); break;
    case 38: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[38])); break;
    case 39: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[39])); break;
    case 40: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[40])); break;
    case 41: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[41])); break;
    case 42: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[42])); break;
    case 43: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[43])); break;
    case 44: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[44])); break;
    case 45: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[45])); break;
    case 46: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[46])); break;
    case 47: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[47])); break;
    case 48: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[48])); break;
    case 49: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[49])); break;
    case 50: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[50])); break;
    case 51: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[51])); break;
    case 52: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[52])); break;
    case 53: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[53])); break;
    case 54: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[54])); break;
    case 55: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[55])); break;
    case 56: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[56])); break;
    case 57: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[57])); break;
    case 58: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[58])); break;
    case 59: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[59])); break;
    case 60: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[60])); break;
    case 61: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[61])); break;
    case 62: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[62])); break;
    case 63: asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[63])); break;
    default: break;
    }
    return v;
}

__device__ __forceinline__ void reg_set64(double (&A)[64], int j, double v) {
    switch (j) {
    case 0: asm("v_mov_b64 %0, %1" : "=v"(A[0]) : "v"(v)); break;
    case 1: asm("v_mov_b64 %0, %1" : "=v"(A[1]) : "v"(v)); break;
    case 2: asm("v_mov_b64 %0, %1" : "=v"(A[2]) : "v"(v)); break;
    case 3: asm("v_mov_b64 %0, %1" : "=v"(A[3]) : "v"(v)); break;
    case 4: asm("v_mov_b64 %0, %1" : "=v"(A[4]) : "v"(v)); break;
    case 5: asm("v_mov_b64 %0, %1" : "=v"(A[5]) : "v"(v)); break;
    case 6: asm("v_mov_b64 %0, %1" : "=v"(A[6]) : "v"(v)); break;
    case 7: asm("v_mov_b64 %0, %1" : "=v"(A[7]) : "v"(v)); break;
    case 8: asm("v_mov_b64 %0, %1" : "=v"(A[8]) : "v"(v)); break;
    case 9: asm("v_mov_b64 %0, %1" : "=v"(A[9]) : "v"(v)); break;
    case 10: asm("v_mov_b64 %0, %1" : "=v"(A[10]) : "v"(v)); break;
    case 11: asm("v_mov_b64 %0, %1" : "=v"(A[11]) : "v"(v)); break;
    case 12: asm("v_mov_b64 %0, %1" : "=v"(A[12]) : "v"(v)); break;
    case 13: asm("v_mov_b64 %0, %1" : "=v"(A[13]) : "v"(v)); break;
    case 14: asm("v_mov_b64 %0, %1" : "=v"(A[14]) : "v"(v)); break;
    case 15: asm("v_mov_b64 %0, %1" : "=v"(A[15]) : "v"(v)); break;
    case 16: asm("v_mov_b64 %0, %1" : "=v"(A[16]) : "v"(v)); break;
    case 17: asm("v_mov_b64 %0, %1" : "=v"(A[17]) : "v"(v)); break;
    case 18: asm("v_mov_b64 %0, %1" : "=v"(A[18]) : "v"(v)); break;
    case 19: asm("v_mov_b64 %0, %1" : "=v"(A[19]) : "v"(v)); break;
    case 20: asm("v_mov_b64 %0, %1" : "=v"(A[20]) : "v"(v)); break;
    case 21: asm("v_mov_b64 %0, %1" : "=v"(A[21]) : "v"(v)); break;
    case 22: asm("v_mov_b64 %0, %1" : "=v"(A[22]) : "v"(v)); break;
    case 23: asm("v_mov_b64 %0, %1" : "=v"(A[23]) : "v"(v)); break;
    case 24: asm("v_mov_b64 %0, %1" : "=v"(A[24]) : "v"(v)); break;
    case 25: asm("v_mov_b64 %0, %1" : "=v"(A[25]) : "v"(v)); break;
    case 26: asm("v_mov_b64 %0, %1" : "=v"(A[26]) : "v"(v)); break;
    case 27: asm("v_mov_b64 %0, %1" : "=v"(A[27]) : "v"(v)); break;
    case 28: asm("v_mov_b64 %0, %1" : "=v"(A[28]) : "v"(v)); break;
    case 29: asm("v_mov_b64 %0, %1" : "=v"(A[29]) : "v"(v)); break;
    case 30: asm("v_mov_b64 %0, %1" : "=v"(A[30]) : "v"(v)); break;
    case 31: asm("v_mov_b64 %0, %1" : "=v"(A[31]) : "v"(v)); break;
    case 32: asm("v_mov_b64 %0, %1" : "=v"(A[32]) : "v"(v)); break;
    case 33: asm("v_mov_b64 %0, %1" : "=v"(A[33]) : "v"(v)); break;
    case 34: asm("v_mov_b64 %0, %1" : "=v"(A[34]) : "v"(v)); break;
    case 35: asm("v_mov_b64 %0, %1" : "=v"(A[35]) : "v"(v)); break;
    case 36: asm("v_mov_b64 %0, %1" : "=v"(A[36]) : "v"(v)); break;
    case 37: asm("v_mov_b64 %0, %1" : "=v"(A[37]) : "v"(v)); break;
    case 38: asm("v_mov_b64 %0, %1" : "=v"(A[38]) : "v"(v)); break;
    case 39: asm("v_mov_b64 %0, %1" : "=v"(A[39]) : "v"(v)); break;
    case 40: asm("v_mov_b64 %0, %1" : "=v"(A[40]) : "v"(v)); break;
    case 41: asm("v_mov_b64 %0, %1" : "=v"(A[41]) : "v"(v)); break;
    case 42: asm("v_mov_b64 %0, %1" : "=v"(A[42]) : "v"(v)); break;
    case 43: asm("v_mov_b64 %0, %1" : "=v"(A[43]) : "v"(v)); break;
    case 44: asm("v_mov_b64 %0, %1" : "=v"(A[44]) : "v"(v)); break;
    case 45: asm("v_mov_b64 %0, %1" : "=v"(A[45]) : "v"(v)); break;
    case 46: asm("v_mov_b64 %0, %1" : "=v"(A[46]) : "v"(v)); break;
    case 47: asm("v_mov_b64 %0, %1" : "=v"(A[47]) : "v"(v)); break;
    case 48: asm("v_mov_b64 %0, %1" : "=v"(A[48]) : "v"(v)); break;
    case 49: asm("v_mov_b64 %0, %1" : "=v"(A[49]) : "v"(v)); break;
    case 50: asm("v_mov_b64 %0, %1" : "=v"(A[50]) : "v"(v)); break;
    case 51: asm("v_mov_b64 %0, %1" : "=v"(A[51]) : "v"(v)); break;
    case 52: asm("v_mov_b64 %0, %1" : "=v"(A[52]) : "v"(v)); break;
    case 53: asm("v_mov_b64 %0, %1" : "=v"(A[53]) : "v"(v)); break;
    case 54: asm("v_mov_b64 %0, %1" : "=v"(A[54]) : "v"(v)); break;
    case 55: asm("v_mov_b64 %0, %1" : "=v"(A[55]) : "v"(v)); break;
    case 56: asm("v_mov_b64 %0, %1" : "=v"(A[56]) : "v"(v)); break;
    case 57: asm("v_mov_b64 %0, %1" : "=v"(A[57]) : "v"(v)); break;
    case 58: asm("v_mov_b64 %0, %1" : "=v"(A[58]) : "v"(v)); break;
    case 59: asm("v_mov_b64 %0, %1" : "=v"(A[59]) : "v"(v)); break;
    case 60: asm("v_mov_b64 %0, %1" : "=v"(A[60]) : "v"(v)); break;
    case 61: asm("v_mov_b64 %0, %1" : "=v"(A[61]) : "v"(v)); break;
    case 62: asm("v_mov_b64 %0, %1" : "=v"(A[62]) : "v"(v)); break;
    case 63: asm("v_mov_b64 %0, %1" : "=v"(A[63]) : "v"(v)); break;
    default: break;
    }
}

// Same contract as gj_invert: A holds A[r][g * 64 + jj] (zero beyond m); on return X
// (column-major, m x m) holds the inverse.  Every thread of the workgroup must call it.
// Partial pivoting without row interchanges: the pivot of column p is the largest
// |a_rp| over rows not yet used (to a relative 2^-13: the search compares the high
// 32 bits of |a_rp|), pi(p) records it, and the stored result S gives
// A^-1[pi^-1(a)][pi(b)] = S[a][b].  Column p is register p & 63 of every thread of
// range g = p >> 6, an index uniform over the workgroup, so it is read and written
// with indexed register moves.  The update is A <- A - (a_rp / a_pp) row with the
// pivot row published with 1 at column p, after which column p is set to
// -a_rp / a_pp (the pivot row starts from 0 with a_rp = -1, giving 1 / a_pp); the
// thread holding a_pp publishes its reciprocal.  The LDS vectors alternate between two
// buffers by the parity of p, so one pivot step needs two barriers.  ds as for gj_invert.
__device__ __forceinline__ void gj_invert64(int m, bool act, int r, int g, double (&A)[64], Gj64Lds& s,
                                            double* X, const double* ds = nullptr) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    bool used = false;
    for (int p = 0; p < m; ++p) {
        const int gp = p >> 6, jp = p & 63, b = p & 1;
        const bool mine = act && g == gp;       // this thread holds column p
        const double pc = reg_get64(A, jp);
        // pivot search key: the high word of |a_rp| with its low 7 bits replaced by
        // 127 - r (largest |a| to 2^-13, then smallest row); 0 for used rows
        unsigned key = 0u;
        if (mine) {
            s.col[b][r] = pc;
            if (!used)
                key = ((unsigned)(__double_as_longlong(fabs(pc)) >> 32) & 0xFFFFFF80u) | (unsigned)(127 - r);
        }
        key = __ockl_wfred_max_u32(key);         // (every lane active here)
        if (lane == 0) s.wk[b][wave] = key;
        __syncthreads();
        unsigned kb = s.wk[b][0];
        for (int w = 1; w < GJ64_T / 64; ++w) kb = max(kb, s.wk[b][w]);
        const int pr = 127 - (int)(kb & 0x7Fu);
        if (t == 0) s.perm[p] = pr;
        const bool piv = act && r == pr;
        if (piv) {          // publish the pivot row (1 at column p), then start it from 0
#pragma unroll
            for (int jj = 0; jj < 64; ++jj) {
                s.row[b][g * 64 + jj] = A[jj];
                A[jj] = 0.0;
            }
            if (g == gp) {
                s.row[b][p] = 1.0;
                s.inv[b] = 1.0 / pc;             // 1 / a_pp, once for the workgroup
            }
            used = true;
        }
        __syncthreads();
        const double crinv = (piv ? -1.0 : s.col[b][r]) * s.inv[b];
        if (act) {
#pragma unroll
            for (int jj = 0; jj < 64; ++jj) A[jj] = fma(-crinv, s.row[b][g * 64 + jj], A[jj]);
            const double v = reg_get64(A, jp);
            reg_set64(A, jp, mine ? -crinv : v);
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
