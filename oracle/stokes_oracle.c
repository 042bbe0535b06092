/*
 * Oracle: plain FP64 brute-force Stokes kernel sums.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the GPU path.
 *
 * Every sum is the definition written out as a double loop over (target,
 * source) pairs, target outer, source inner, in FP64 with sqrt and divisions.
 * No blocking, no reordering, no precomputed source quantities.
 *
 * Arrays are structure-of-arrays: a point set of n points is three planes
 * x[0..n), y[0..n), z[0..n) stored back to back (index c*n + i).
 *
 * Paper: Nazockdast, Rahimian, Zorin, Shelley, arXiv:1602.05650.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double ORACLE_PI = 3.14159265358979323846264338327950288;

/*
 * Single layer over fiber nodes: Stokeslet plus source doublet.
 *
 *   u(x_i) = sum_{j not excluded}  w_j [ G(d) f_j + c_j W(d) f_j ],   d = x_i - y_j
 *
 *   G(d) f = (1/(8 pi mu)) ( f/|d| + d (d.f)/|d|^3 )            (section 2, eq. oseen,
 *                                                                 applied in eq. single-layer)
 *   W(d) f = (1/(8 pi mu)) ( f/|d|^3 - 3 d (d.f)/|d|^5 )          (eq. main-sb-vel, doublet)
 *   c_j    = a_j^2 / 2,  a_j = eps * L_{fiber(j)}                  (eq. main-sb-vel: the eps^2/2
 *                                                                 factor, with eps = a/L)
 *
 * Exclusion (excl):
 *   0  none
 *   1  the target's own point: j == self(i)           (self-pairs excluded)
 *   2  the target's own fiber: fiber(j) == fiber(i)   (eq. complementary-uf, l != m)
 * self(i) = tself[i] if given, else i when the targets are the sources, else none.
 * fiber(i) = tfib[i] if given, else sfib[i] when the targets are the sources.
 *
 * weights w: NULL means 1.  flen: per-fiber length, NULL means 1.  sfib NULL
 * means every source is a fiber of length flen[0] (or 1).
 * A pair with |d| == 0 that is not excluded contributes nothing and is counted.
 * Returns that count.
 */
int64_t oracle_sl(int64_t ns, const double* sx, const double* f, const double* w,
                  const int32_t* sfib, const double* flen,
                  int64_t nt, const double* tx, const int64_t* tself, const int32_t* tfib,
                  double mu, double eps, int excl, int doublet, double* u, int nthreads)
{
    const int targets_are_sources = (tx == NULL);
    const double* X = targets_are_sources ? sx : tx;
    const int64_t ntt = targets_are_sources ? ns : nt;
    const double pref = 1.0 / (8.0 * ORACLE_PI * mu);
    int64_t skipped = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+:skipped) if(nthreads != 1)
#endif
    for (int64_t i = 0; i < ntt; ++i) {
        const double xi = X[i], yi = X[ntt + i], zi = X[2 * ntt + i];
        int64_t self = -1;
        if (tself) self = tself[i];
        else if (targets_are_sources) self = i;
        int64_t fib_i = -1;
        if (tfib) fib_i = tfib[i];
        else if (targets_are_sources && sfib) fib_i = sfib[i];
        double ux = 0.0, uy = 0.0, uz = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            if (excl == 1 && j == self) continue;
            if (excl == 2 && sfib && (int64_t)sfib[j] == fib_i) continue;
            const double dx = xi - sx[j];
            const double dy = yi - sx[ns + j];
            const double dz = zi - sx[2 * ns + j];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) { skipped += 1; continue; }
            const double r = sqrt(r2);
            const double wj = w ? w[j] : 1.0;
            const double fx = wj * f[j], fy = wj * f[ns + j], fz = wj * f[2 * ns + j];
            const double df = dx * fx + dy * fy + dz * fz;
            const double r3 = r2 * r;
            /* Stokeslet: f/r + d (d.f)/r^3 */
            double gx = fx / r + dx * df / r3;
            double gy = fy / r + dy * df / r3;
            double gz = fz / r + dz * df / r3;
            if (doublet) {
                double L = 1.0;
                if (flen) L = sfib ? flen[sfib[j]] : flen[0];
                const double a = eps * L;
                const double c = 0.5 * a * a;
                const double r5 = r3 * r2;
                /* doublet: f/r^3 - 3 d (d.f)/r^5 */
                gx += c * (fx / r3 - 3.0 * dx * df / r5);
                gy += c * (fy / r3 - 3.0 * dy * df / r5);
                gz += c * (fz / r3 - 3.0 * dz * df / r5);
            }
            ux += gx; uy += gy; uz += gz;
        }
        u[i] = pref * ux;
        u[ntt + i] = pref * uy;
        u[2 * ntt + i] = pref * uz;
    }
    return skipped;
}

/*
 * Double layer over surface quadrature points (stresslet).
 *
 *   u(x_i) = (3/(4 pi)) sum_{s != self(i)} w_s (d . qt_s)(d . n_s) d / |d|^5,   d = x_i - y_s
 *
 * This is eq. double-layer with the stresslet of eq. stresslet, the viscosity
 * dropped (the density q is a velocity) and the sign taken so that, with the
 * outward normal n, a constant density q gives -q inside the surface, 0
 * outside and -q/2 (principal value) on it, the convention under which the
 * periphery equation main-cortex-density reads -q/2 + T[q] + N[q] = -u_bar.
 *
 * subtract = 1 (on-surface singularity subtraction, section "Singular
 * integrals over surfaces"): for a target with self(i) >= 0,
 * qt_s = q_s - q_{self(i)} and afterwards -q_{self(i)}/2 is added, which gives
 * the principal value; off-surface targets (self < 0) use qt_s = q_s.
 * subtract = 0: qt_s = q_s and the self point is simply left out.
 * self(i) = tself[i] if given, else i when the targets are the surface points.
 * A pair with |d| == 0 that is not the self pair is skipped and counted.
 */
int64_t oracle_dl(int64_t ns, const double* sx, const double* n, const double* w, const double* q,
                  int64_t nt, const double* tx, const int64_t* tself, int subtract,
                  double* u, int nthreads)
{
    const int targets_are_sources = (tx == NULL);
    const double* X = targets_are_sources ? sx : tx;
    const int64_t ntt = targets_are_sources ? ns : nt;
    const double pref = 3.0 / (4.0 * ORACLE_PI);
    int64_t skipped = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+:skipped) if(nthreads != 1)
#endif
    for (int64_t i = 0; i < ntt; ++i) {
        const double xi = X[i], yi = X[ntt + i], zi = X[2 * ntt + i];
        int64_t self = -1;
        if (tself) self = tself[i];
        else if (targets_are_sources) self = i;
        double q0x = 0.0, q0y = 0.0, q0z = 0.0;
        const int sub = subtract && self >= 0 && self < ns;
        if (sub) { q0x = q[self]; q0y = q[ns + self]; q0z = q[2 * ns + self]; }
        double ux = 0.0, uy = 0.0, uz = 0.0;
        for (int64_t s = 0; s < ns; ++s) {
            if (s == self) continue;
            const double dx = xi - sx[s];
            const double dy = yi - sx[ns + s];
            const double dz = zi - sx[2 * ns + s];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) { skipped += 1; continue; }
            const double r = sqrt(r2);
            const double r5 = r2 * r2 * r;
            const double qx = q[s] - q0x, qy = q[ns + s] - q0y, qz = q[2 * ns + s] - q0z;
            const double dq = dx * qx + dy * qy + dz * qz;
            const double dn = dx * n[s] + dy * n[ns + s] + dz * n[2 * ns + s];
            const double k = w[s] * dq * dn / r5;
            ux += k * dx; uy += k * dy; uz += k * dz;
        }
        ux *= pref; uy *= pref; uz *= pref;
        if (sub) { ux -= 0.5 * q0x; uy -= 0.5 * q0y; uz -= 0.5 * q0z; }
        u[i] = ux;
        u[ntt + i] = uy;
        u[2 * ntt + i] = uz;
    }
    return skipped;
}

int oracle_has_openmp(void)
{
#ifdef _OPENMP
    return 1;
#else
    return 0;
#endif
}
