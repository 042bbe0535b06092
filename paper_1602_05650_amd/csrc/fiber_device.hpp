// Device helpers of the fiber operators shared by the mobility solve and the
// implicit time step: Clenshaw-Curtis weights on the CGL nodes, the local
// slender-body operator M (and its inverse), and the nonlocal self term K_delta.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stokes {

// Clenshaw-Curtis weight of node kk on the p+1 CGL nodes cos(k pi/p) (Waldvogel's
// closed form): w_k = (c_k/p) (1 - sum_{j=1}^{p/2} b_j cos(2 j k pi/p) / (4 j^2 - 1)).
__device__ inline double cc_weight(int kk, int p) {
    if (p == 1) return 1.0;
    double s = 0.0;
    for (int j = 1; j <= p / 2; ++j) {
        const double b = (2 * j == p) ? 1.0 : 2.0;
        s += b * cos(2.0 * j * kk * 3.14159265358979323846 / p) / (4.0 * j * j - 1.0);
    }
    const double c = (kk == 0 || kk == p) ? 1.0 : 2.0;
    return c / p * (1.0 - s);
}

// out = a f + b t (t.f): M (inverse = 0) or M^{-1} (inverse = 1), eq. main-sb-local.
__device__ __forceinline__ void apply_local(double kap, double mu, bool inverse, double tx,
                                            double ty, double tz, double& fx, double& fy,
                                            double& fz) {
    const double pi8mu = 8.0 * 3.14159265358979323846 * mu;
    double a, b;
    if (!inverse) {
        a = (kap + 2.0) / pi8mu;
        b = (kap - 2.0) / pi8mu;
    } else {
        a = pi8mu / (kap + 2.0);
        b = pi8mu / (2.0 * kap) - a;
    }
    const double tf = tx * fx + ty * fy + tz * fz;
    fx = a * fx + b * tf * tx;
    fy = a * fy + b * tf * ty;
    fz = a * fz + b * tf * tz;
}

// K_delta[f] at node i (eq. sb-stokes-reg) over the other nodes of its fiber, with
// the fiber's quadrature weights wq and arc lengths sarc.  |r|/sqrt(r^2+d^2) G(r) f_k
// is written (f_k + r (r.f_k)/r^2) / (8 pi mu sqrt(r^2 + d^2)).
__device__ inline void nonlocal_at(int64_t i, int64_t N, int npf, const double* xyz, const double* tan,
                            const double* f, const double* wq, const double* sarc, double delta,
                            double pref, double& ox, double& oy, double& oz) {
    const int64_t f0 = (i / npf) * npf;
    const double xi = xyz[i], yi = xyz[N + i], zi = xyz[2 * N + i];
    const double si = sarc[i], d2 = delta * delta;
    double ax = 0.0, ay = 0.0, az = 0.0, dsum = 0.0;
    for (int k = 0; k < npf; ++k) {
        const int64_t j = f0 + k;
        if (j == i) continue;
        const double rx = xi - xyz[j], ry = yi - xyz[N + j], rz = zi - xyz[2 * N + j];
        const double fx = f[j], fy = f[N + j], fz = f[2 * N + j];
        const double r2 = rx * rx + ry * ry + rz * rz;
        const double a = wq[j] / sqrt(r2 + d2);
        const double b = a * (rx * fx + ry * fy + rz * fz) / r2;
        ax += a * fx + b * rx;
        ay += a * fy + b * ry;
        az += a * fz + b * rz;
        const double ds = si - sarc[j];
        dsum += wq[j] / sqrt(ds * ds + d2);
    }
    const double tx = tan[i], ty = tan[N + i], tz = tan[2 * N + i];
    const double fx = f[i], fy = f[N + i], fz = f[2 * N + i];
    const double tf = tx * fx + ty * fy + tz * fz;
    ox = pref * (ax - dsum * (fx + tf * tx));
    oy = pref * (ay - dsum * (fy + tf * ty));
    oz = pref * (az - dsum * (fz + tf * tz));
}

}  // namespace stokes
