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

// Register j of A for an index j uniform over the wave: a switch on j (scalar
// branches) around one register move per case.  The moves are written as inline asm
// so that the cases cannot be folded into an indexed access, which would move A to
// scratch memory.  NC <= 64.
#define STOKES_REG_CASES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) \
    X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) \
    X(30) X(31) X(32) X(33) X(34) X(35) X(36) X(37) X(38) X(39) X(40) X(41) X(42) X(43) \
    X(44) X(45) X(46) X(47) X(48) X(49) X(50) X(51) X(52) X(53) X(54) X(55) X(56) X(57) \
    X(58) X(59) X(60) X(61) X(62) X(63)

template <int NC>
__device__ __forceinline__ double reg_get(const double (&A)[NC], int j) {
    static_assert(NC <= 64, "at most 64 registers");
    double v = 0.0;
    switch (j) {
#define STOKES_GET(k) \
    case k:                                                            \
        if constexpr (k < NC) asm("v_mov_b64 %0, %1" : "=v"(v) : "v"(A[k])); \
        break;
        STOKES_REG_CASES(STOKES_GET)
#undef STOKES_GET
    default: break;
    }
    return v;
}

template <int NC>
__device__ __forceinline__ void reg_set(double (&A)[NC], int j, double v) {
    static_assert(NC <= 64, "at most 64 registers");
    switch (j) {
#define STOKES_SET(k) \
    case k:                                                            \
        if constexpr (k < NC) asm("v_mov_b64 %0, %1" : "=v"(A[k]) : "v"(v)); \
        break;
        STOKES_REG_CASES(STOKES_SET)
#undef STOKES_SET
    default: break;
    }
}
#undef STOKES_REG_CASES

struct GjLds {
    double col[2][GJ_MAX], row[2][GJ_MAX], inv[2];
    unsigned wk[2][BLOCK_GJ / 64];
    int perm[GJ_MAX], dest[GJ_MAX];
};

// A holds this thread's entries A[r][g + GJ_G jj] on entry (zero where the thread is
// inactive or the column is >= m).  On return X (column-major, m x m) holds the
// inverse; a singular matrix gives a result that is not finite.  Every thread of the
// workgroup must call it.  (act, r, g) are the thread's role as set out above:
// act = t < GJ_G m, r = t % m, g = t / m (both 0 when inactive).
// ds (LDS or null): the result's column j is multiplied by ds[j] (the inverse of a
// row-equilibrated matrix D B gives B^-1 = (D B)^-1 D).
// Partial pivoting without row interchanges: the pivot of column p is the largest
// |a_rp| over rows not yet used (to a relative 2^-12: the search compares the high
// 32 bits of |a_rp|, its low 8 bits replaced by 255 - r so that ties go to the
// smallest row), pi(p) records it, and the stored result S gives
// A^-1[pi^-1(a)][pi(b)] = S[a][b].  Column p is register p / GJ_G of the threads with
// g = p % GJ_G, an index uniform over the workgroup (see reg_get).  The update is
// A <- A - (a_rp / a_pp) row, after which column p is set to -a_rp / a_pp (the pivot
// row starts from 0 with a_rp = -1, giving 1 / a_pp); the thread holding a_pp
// publishes its reciprocal.  The LDS vectors
// alternate between two buffers by the parity of p, so one pivot step needs two
// barriers.
__device__ __forceinline__ void gj_invert(int m, bool act, int r, int g, double (&A)[GJ_COLS], GjLds& s,
                                          double* X, const double* ds = nullptr) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    bool used = false;
    for (int p = 0; p < m; ++p) {
        const int gp = p % GJ_G, jp = p / GJ_G, b = p & 1;
        const bool mine = act && g == gp;       // this thread holds column p
        const double pc = reg_get(A, jp);
        unsigned key = 0u;
        if (mine) {
            s.col[b][r] = pc;
            if (!used)
                key = ((unsigned)(__double_as_longlong(fabs(pc)) >> 32) & 0xFFFFFF00u) | (unsigned)(255 - r);
        }
        key = __ockl_wfred_max_u32(key);         // (every lane active here)
        if (lane == 0) s.wk[b][wave] = key;
        __syncthreads();
        unsigned kb = s.wk[b][0];
        for (int w = 1; w < BLOCK_GJ / 64; ++w) kb = max(kb, s.wk[b][w]);
        const int pr = 255 - (int)(kb & 0xFFu);
        if (t == 0) s.perm[p] = pr;
        const bool piv = act && r == pr;
        if (piv) {          // publish the pivot row, then start it from 0
#pragma unroll
            for (int jj = 0; jj < GJ_COLS; ++jj) {
                const int c = g + GJ_G * jj;
                if (c < m) s.row[b][c] = A[jj];
                A[jj] = 0.0;
            }
            if (g == gp) s.inv[b] = 1.0 / pc;   // 1 / a_pp, once for the workgroup
            used = true;
        }
        __syncthreads();
        const double crinv = (piv ? -1.0 : s.col[b][r]) * s.inv[b];
        if (act) {
#pragma unroll
            for (int jj = 0; jj < GJ_COLS; ++jj) {
                const int c = g + GJ_G * jj;
                if (c < m) A[jj] = fma(-crinv, s.row[b][c], A[jj]);
            }
            const double v = reg_get(A, jp);
            reg_set(A, jp, mine ? -crinv : v);
        }
    }
    __syncthreads();
    if (t == 0)
        for (int p = 0; p < m; ++p) s.dest[s.perm[p]] = p;     // pi^-1
    __syncthreads();
    if (act) {
        const int row_out = s.dest[r];
#pragma unroll
        for (int jj = 0; jj < GJ_COLS; ++jj) {
            const int c = g + GJ_G * jj;
            if (c < m) X[(int64_t)s.perm[c] * m + row_out] = ds ? A[jj] * ds[s.perm[c]] : A[jj];
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

struct alignas(16) Gj64Lds {   // (16-byte aligned: the pivot row is read as double2)
    double col[2][GJ64_MAX], row[2][GJ64_MAX], inv[2];
    unsigned wk[2][GJ64_T / 64];
    int perm[GJ64_MAX], dest[GJ64_MAX];
};

// Same contract as gj_invert: A holds A[r][g * 64 + jj] (zero beyond m); on return X
// (column-major, m x m) holds the inverse.  Every thread of the workgroup must call it.
// Partial pivoting without row interchanges: the pivot of column p is the largest
// |a_rp| over rows not yet used (to a relative 2^-13: the search compares the high
// 32 bits of |a_rp|), pi(p) records it, and the stored result S gives
// A^-1[pi^-1(a)][pi(b)] = S[a][b].  Column p is register p & 63 of every thread of
// range g = p >> 6, an index uniform over the workgroup, so it is read and written
// with indexed register moves.  The update is A <- A - (a_rp / a_pp) row, after
// which column p is set to -a_rp / a_pp (the pivot row starts from 0 with a_rp = -1,
// giving 1 / a_pp); the thread holding a_pp publishes its reciprocal.  The LDS vectors alternate between two
// buffers by the parity of p, so one pivot step needs two barriers.  ds as for gj_invert.
__device__ __forceinline__ void gj_invert64(int m, bool act, int r, int g, double (&A)[64], Gj64Lds& s,
                                            double* X, const double* ds = nullptr) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    bool used = false;
    for (int p = 0; p < m; ++p) {
        const int gp = p >> 6, jp = p & 63, b = p & 1;
        const bool mine = act && g == gp;       // this thread holds column p
        const double pc = reg_get(A, jp);
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
        if (piv) {          // publish the pivot row, then start it from 0
#pragma unroll
            for (int jj = 0; jj < 64; ++jj) {
                s.row[b][g * 64 + jj] = A[jj];
                A[jj] = 0.0;
            }
            if (g == gp) s.inv[b] = 1.0 / pc;   // 1 / a_pp, once for the workgroup
            used = true;
        }
        __syncthreads();
        const double crinv = (piv ? -1.0 : s.col[b][r]) * s.inv[b];
        if (act) {
#pragma unroll
            for (int jb = 0; jb < 64; jb += 16) {   // the pivot row in blocks of 16 (loads in flight together)
                const double2* src = reinterpret_cast<const double2*>(&s.row[b][g * 64 + jb]);
                double2 rv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) rv[q] = src[q];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    A[jb + 2 * q] = fma(-crinv, rv[q].x, A[jb + 2 * q]);
                    A[jb + 2 * q + 1] = fma(-crinv, rv[q].y, A[jb + 2 * q + 1]);
                }
            }
            const double v = reg_get(A, jp);
            reg_set(A, jp, mine ? -crinv : v);
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
