// Device arithmetic shared by the direct sums (sum_device.hpp) and the treecode
// (stokes_tree.hip): the FP64 reciprocal square root and the tangent band of a run
// of double-layer sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stokes {

// 1/sqrt(x) to full FP64 accuracy for x > 0: the hardware estimate y (about 2^-24
// relative on gfx950), then one third-order Newton-Raphson step
// y (1 + e/2 + 3 e^2/8), e = 1 - x y^2.
__device__ __forceinline__ double rsqrt64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    const double e = fma(-h, y, 1.0);
    const double p = fma(e, 0.375, 0.5);
    return fma(y * e, p, y);
}

// |d|^-5 in FP32 from r2 = |d|^2 and ri ~ rsq(r2) (0 for a masked pair: gives 0).
// The hardware estimate's error, multiplied by five in ri^5 and not centred on zero,
// would scale the whole stresslet by a common factor; on the surface the subtracted
// sum is ~ q_self / 2 while the result is a few hundredths of that, so a bias of one
// ulp in rsq gave 2e-5 relative error in FP32 models.  One Newton correction removes
// it: with e = 1 - r2 ri^2 (exact product in the FMA), ri^5 (1 + 5e/2) leaves only
// round-to-nearest errors.
__device__ __forceinline__ float rinv5_f32(float r2, float ri) {
    const float ri2 = ri * ri;
    const float ri5 = ri2 * ri2 * ri;
    const float e = fmaf(-r2, ri2, 1.0f);
    return fmaf(ri5, 2.5f * e, ri5);
}

// Tangent band of the double layer's mixed path: the radius within which the stresslet
// pairs of a run of surface sources need d and d.n in FP64.  For a target on or near a
// smooth surface d is nearly tangent to it, and d.n ~ |d|^2 / (2 R_curv); formed in FP32
// (rounded coordinates, rounded normal, rounded dot product) it carries a relative error
// ~ eps32 2 R_curv / |d|.  Summed over the pairs beyond a radius rho this gives a
// relative error of the result ~ eps32 R_curv / rho, which does not fall as the surface
// is refined.  The band is BAND_CURV times the run's smallest curvature radius,
// estimated by chords from two of its points (the first and the middle one) to the
// others: min |y_j - y_k| / |n_j - n_k|, exactly R on a sphere of radius R.  A flat run
// gets an unbounded band.  FP32 models of the mixed sum with this band, on spheres of
// 6,144 to 393,216 points carrying a random density (subtracted; the principal value's
// cancellation leaves |u| at 0.01-0.08 of |q|), gave 1.2e-6 to 1.5e-6 relative max-norm
// error, against 5e-6 to 2.5e-5 with FP32 d.n everywhere.
constexpr double BAND_CURV = 0.1;
constexpr double BAND_MAX = 1e15;

// Run [j0, j1) of sources with positions x[c * ld + j] and normals n[c * ld + j];
// UNIT false: the normals carry a positive weight (w n) and are normalised here.
template <bool UNIT = true>
__device__ __forceinline__ double dl_band_radius(int64_t j0, int64_t j1, int64_t ld,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ n) {
    double k2 = 0.0;   // largest |dn|^2 / |dy|^2 over the chords
    const int64_t jm = (j0 + j1) / 2;
    for (int64_t j = j0; j <= jm; j += (jm - j0 > 0 ? jm - j0 : 1)) {
        double nj[3], sj = 1.0;
        for (int c = 0; c < 3; ++c) nj[c] = n[c * ld + j];
        if (!UNIT) sj = 1.0 / sqrt(nj[0] * nj[0] + nj[1] * nj[1] + nj[2] * nj[2]);
        for (int64_t k = j0; k < j1; ++k) {
            double nk[3], sk = 1.0;
            for (int c = 0; c < 3; ++c) nk[c] = n[c * ld + k];
            if (!UNIT) sk = 1.0 / sqrt(nk[0] * nk[0] + nk[1] * nk[1] + nk[2] * nk[2]);
            double dy2 = 0.0, dn2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double dy = x[c * ld + j] - x[c * ld + k];
                const double dn = nj[c] * sj - nk[c] * sk;
                dy2 += dy * dy;
                dn2 += dn * dn;
            }
            if (dy2 > 0.0) k2 = fmax(k2, dn2 / dy2);
        }
    }
    return k2 > 0.0 ? fmin(BAND_CURV / sqrt(k2), BAND_MAX) : BAND_MAX;
}

// dl_band_radius<true> of the run [j0, j1) by the 32 lanes of a half-wave (lane l takes
// point j0 + l against the first and the middle point): the same chords, the same max.
__device__ __forceinline__ double dl_band_radius_half(int l, int64_t j0, int64_t j1, int64_t ld,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ n) {
    const int64_t jm = (j0 + j1) / 2;
    const int64_t k = j0 + l;
    double k2 = 0.0;
    if (k < j1) {
        for (int64_t j = j0; j <= jm; j += (jm - j0 > 0 ? jm - j0 : 1)) {
            double dy2 = 0.0, dn2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double dy = x[c * ld + j] - x[c * ld + k];
                const double dn = n[c * ld + j] - n[c * ld + k];
                dy2 += dy * dy;
                dn2 += dn * dn;
            }
            if (dy2 > 0.0) k2 = fmax(k2, dn2 / dy2);
        }
    }
    for (int off = 16; off > 0; off >>= 1) k2 = fmax(k2, __shfl_xor(k2, off, 32));
    return k2 > 0.0 ? fmin(BAND_CURV / sqrt(k2), BAND_MAX) : BAND_MAX;
}

}  // namespace stokes
