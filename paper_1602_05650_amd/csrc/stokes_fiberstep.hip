// One implicit (backward Euler) time step of free elastic fibers (section "Time
// discretization"), solved on the device by right-preconditioned FP64 GMRES.
//
// Unknowns per fiber (n = p + 1 CGL nodes, node 0 at s = L): the increment
// dX = X+ - X (3 n) and the tension T+ (n).  With s = 2 / L, the force
//   f = -E s^4 D4 X+ + s D1 (T+ X_s)                                  (X_s = s X_a)
// and the velocity V[f] = A f + R[f]: A = alpha I + beta t t acts node by node (M, and
// with the nonlocal term the subtracted local part of K_delta), R is the rest of
// K_delta and the other fibers' Stokeslet + doublet sum (Clenshaw-Curtis weights x
// L/2).  The rows are
//   position   P4 (X+ / dt - V[f+]) = P4 (X / dt + V[f_ext])    (n - 4 per component)
//              X+_ss = 0, X+_sss = 0 at s = L and s = 0          (eq. bc-free)
//   tension    -P2 (h(X+, T+) + t . D_s R[f+]) = P2 t . D_s V[f_ext]   (n - 2)
//              T+ = 0 at both ends
// where h = c_s (t . f+) + c (t . f+)_s - alpha X_ss . f+ (c = alpha + beta) is t . (A f+)_s
// with the arclength identities: t . f+ = 3 E X_ss . X+_sss + T_s,
// (t . f+)_s = 3 E (X_sss . X+_sss + X_ss . X+_ssss) + T_ss, X_ss . f+ = -E X_ss . X+_ssss
// + |X_ss|^2 T (the velocity form of eq. main-inextensibility as a second-order
// equation for T).  P4 and P2 resample node values to n - 4 and n - 2 first-kind
// Chebyshev points (rectangular collocation).  Written for the increment, the
// right-hand side gains the same rows applied to the current nodes.
//
// Layout of every vector of the solve: [dX_x (N) | dX_y (N) | dX_z (N) | T (N)],
// padded with zeros to the Krylov slot's 3 n_vec entries; the rows of fiber f sit
// at the same places (position rows c N + f n + j, tension rows 3 N + f n + j).
// Preconditioner: per fiber the rows without the other fibers' flow, a dense
// 4n x 4n block built on the device and inverted by Gauss-Jordan (gj_device.hpp).
#include <math.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "cheb_tables.hpp"
#include "fiber_device.hpp"
#include "gj_device.hpp"
#include "solver_batch.hpp"

namespace stokes {
namespace fs {

constexpr int EB = 256;           // elementwise kernels
constexpr int FB = 256;           // per-fiber kernels
constexpr int MAX_NPF = GJ_MAX / 4;
constexpr int PREP_CHUNK = 512;   // fibers per pass of the block set-up

struct Geo {
    int64_t N;
    int n, nf;
    const double* X;      // [3N] current nodes
    const double* flen;   // [nf]
    const double* Xa;     // [3N] D1 X
    const double* tan;    // [3N] unit tangents
    const double* wq;     // [N] Clenshaw-Curtis weights x L/2
    const double* sarc;   // [N] arclength of the nodes
    const double* xss;    // [3N] X_ss, X_sss of the current nodes
    const double* xsss;
    const double* alpha;  // [N] A = alpha I + (c - alpha) t t; c_s = D_s c
    const double* cc;
    const double* cs;
    const double* D1;     // n x n tables (row-major)
    const double* D2;
    const double* D3;
    const double* D4;
    const double* P4;     // (n - 4) x n
    const double* P2;     // (n - 2) x n
    const int32_t* clamp; // [nf] or null: minus end 0 free, 2 hinged, other: clamped (body at rest)
    double E, dt, mu, kappa, pref, delta;
    bool nonlocal;
};

// minus-end condition of fiber f: 0 free, 1 clamped, 2 hinged
__device__ __forceinline__ int end_kind(const Geo& g, int f) {
    const int v = g.clamp ? g.clamp[f] : 0;
    return v == 0 ? 0 : (v == 2 ? 2 : 1);
}

__global__ __launch_bounds__(EB) void k_fs_geom(Geo g, double* Xa, double* tan, double* wq,
                                                double* sarc, int32_t* fib, double* xss, double* xsss,
                                                double* alpha, double* cc) {
    const int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (i >= g.N) return;
    const int n = g.n, p = n - 1, f = (int)(i / n), kk = (int)(i - (int64_t)f * n);
    const int64_t f0 = (int64_t)f * n, N = g.N;
    const double L = g.flen[f], s = 2.0 / L;
    double a[3];
    for (int c = 0; c < 3; ++c) {   // D_k (X - X_0): the same derivatives without the offset's rounding
        const double* xc = g.X + c * N + f0;
        double d1 = 0.0, d2 = 0.0, d3 = 0.0;
        for (int k = 0; k < n; ++k) {
            const double x = xc[k] - xc[0];
            d1 = fma(g.D1[kk * n + k], x, d1);
            d2 = fma(g.D2[kk * n + k], x, d2);
            d3 = fma(g.D3[kk * n + k], x, d3);
        }
        a[c] = d1;
        xss[c * N + i] = s * s * d2;
        xsss[c * N + i] = s * s * s * d3;
    }
    const double inv = 1.0 / sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int c = 0; c < 3; ++c) {
        Xa[c * N + i] = a[c];
        tan[c * N + i] = a[c] * inv;
    }
    const double PI = 3.14159265358979323846;
    const double si = 0.5 * L * (1.0 + cos(kk * PI / p));
    wq[i] = cc_weight(kk, p) * 0.5 * L;
    sarc[i] = si;
    fib[i] = f;
    double dsum = 0.0;
    if (g.nonlocal) {
        const double d2 = g.delta * g.delta;
        for (int q = 0; q < n; ++q) {
            if (q == kk) continue;
            const double ds = si - 0.5 * L * (1.0 + cos(q * PI / p));
            dsum += cc_weight(q, p) * 0.5 * L / sqrt(ds * ds + d2);
        }
    }
    alpha[i] = g.pref * (g.kappa + 2.0 - dsum);
    cc[i] = g.pref * (2.0 * g.kappa - 2.0 * dsum);
}

__global__ __launch_bounds__(EB) void k_fs_geom2(Geo g, double* cs) {
    const int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (i >= g.N) return;
    const int n = g.n, f = (int)(i / n), kk = (int)(i - (int64_t)f * n);
    const int64_t f0 = (int64_t)f * n;
    double d = 0.0;
    for (int k = 0; k < n; ++k) d = fma(g.D1[kk * n + k], g.cc[f0 + k], d);
    cs[i] = 2.0 / g.flen[f] * d;
}

// f = -E s^4 D4 zX + s D1 (zT X_s) (+ fext).  zT may be null (no tension term).  D4 acts
// on zX minus the fiber's first node (D4 of a constant is zero): for zX = X this keeps
// rounding proportional to the fiber's extent instead of its distance from the origin.
__global__ __launch_bounds__(EB) void k_fs_force(Geo g, const double* zX, const double* zT,
                                                 const double* fext, double* f) {
    const int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (i >= g.N) return;
    const int n = g.n, fi = (int)(i / n), kk = (int)(i - (int64_t)fi * n);
    const int64_t f0 = (int64_t)fi * n, N = g.N;
    const double s = 2.0 / g.flen[fi], e4 = -g.E * s * s * s * s;
    const double* d4 = g.D4 + kk * n;
    const double* d1 = g.D1 + kk * n;
    for (int c = 0; c < 3; ++c) {
        const double ref = zX[c * N + f0];
        double b = 0.0, t = 0.0;
        for (int k = 0; k < n; ++k) {
            b = fma(d4[k], zX[c * N + f0 + k] - ref, b);
            if (zT) t = fma(d1[k], zT[f0 + k] * g.Xa[c * N + f0 + k], t);
        }
        double v = e4 * b + s * s * t;
        if (fext) v += fext[c * N + i];
        f[c * N + i] = v;
    }
}

// vr = K_delta f + (local part of K_delta, added back) at every node, or zero: the
// smooth part R of the velocity before the other fibers' flow is added in.
__global__ __launch_bounds__(EB) void k_fs_smooth(Geo g, const double* f, double* vr) {
    const int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (i >= g.N) return;
    const int64_t N = g.N;
    double x = 0.0, y = 0.0, z = 0.0;
    if (g.nonlocal) {
        nonlocal_at(i, N, g.n, g.X, g.tan, f, g.wq, g.sarc, g.delta, g.pref, x, y, z);
        // local part -(pref dsum)(I + t t) f with pref dsum = (alpha_M - alpha)
        const double pd = g.pref * (g.kappa + 2.0) - g.alpha[i];
        const double tx = g.tan[i], ty = g.tan[N + i], tz = g.tan[2 * N + i];
        const double fx = f[i], fy = f[N + i], fz = f[2 * N + i];
        const double tf = tx * fx + ty * fy + tz * fz;
        x += pd * (fx + tf * tx);
        y += pd * (fy + tf * ty);
        z += pd * (fz + tf * tz);
    }
    vr[i] = x;
    vr[N + i] = y;
    vr[2 * N + i] = z;
}

// The rows of one fiber per workgroup.  rhs = false: the operator on z with f = F z and
// vr = R[f].  rhs = true: the right-hand side with f = f_ext - E s^4 D4 X, vr = R[f],
// fe = f_ext, and the current nodes in the place of z (boundary defects, h(X, 0)).
constexpr int ROWS_FPB = 4;   // fibers per workgroup of k_fs_rows (64 threads each)
__global__ __launch_bounds__(64 * ROWS_FPB) void k_fs_rows(Geo g, const double* z, const double* f,
                                                           const double* vr, const double* fe, bool rhs,
                                                           double* w) {
    __shared__ double pk_all[ROWS_FPB][3][MAX_NPF], hk_all[ROWS_FPB][MAX_NPF], cl_all[ROWS_FPB];
    const int n = g.n, fl = threadIdx.x / 64, t = threadIdx.x % 64;
    const int fi = blockIdx.x * ROWS_FPB + fl;
    const bool live = fi < g.nf;
    double(*pk)[MAX_NPF] = pk_all[fl];
    double* hk = hk_all[fl];
    const int64_t N = g.N, f0 = (int64_t)(live ? fi : 0) * n;
    const double s = 2.0 / g.flen[live ? fi : 0], E = g.E;
    if (live && t < n) {
        const int64_t i = f0 + t;
        const double* d1 = g.D1 + t * n;
        const double* d2 = g.D2 + t * n;
        const double* d3 = g.D3 + t * n;
        const double* d4 = g.D4 + t * n;
        const double al = g.alpha[i], be = g.cc[i] - al;
        double tv[3], ssf = 0.0, ss3 = 0.0, ss4 = 0.0, sss3 = 0.0, tdv = 0.0, tdl = 0.0;
        for (int c = 0; c < 3; ++c) tv[c] = g.tan[c * N + i];
        double tfv = 0.0;
        for (int c = 0; c < 3; ++c) tfv = fma(tv[c], f[c * N + i], tfv);
        for (int c = 0; c < 3; ++c) {
            const double* zc = z + c * N + f0;
            const double* vc = vr + c * N + f0;
            double x3 = 0.0, x4 = 0.0, dv = 0.0, dl = 0.0;
            for (int k = 0; k < n; ++k) {
                const double zk = zc[k] - zc[0];
                x3 = fma(d3[k], zk, x3);
                x4 = fma(d4[k], zk, x4);
                dv = fma(d1[k], vc[k], dv);
                if (rhs) {   // D1 (A f_ext): the local velocity of the external force
                    const int64_t j = f0 + k;
                    const double ak = g.alpha[j], bk = g.cc[j] - ak;
                    const double tj = g.tan[c * N + j];
                    double tfe_k = 0.0;
                    for (int e = 0; e < 3; ++e) tfe_k = fma(g.tan[e * N + j], fe[e * N + j], tfe_k);
                    dl = fma(d1[k], ak * fe[c * N + j] + bk * tj * tfe_k, dl);
                }
            }
            x3 *= s * s * s;
            x4 *= s * s * s * s;
            const double xs2 = g.xss[c * N + i], xs3 = g.xsss[c * N + i];
            ss3 = fma(xs2, x3, ss3);
            ss4 = fma(xs2, x4, ss4);
            sss3 = fma(xs3, x3, sss3);
            tdv = fma(tv[c], s * dv, tdv);
            tdl = fma(tv[c], s * dl, tdl);
            const double av = al * f[c * N + i] + be * tv[c] * tfv + vr[c * N + i];   // V[f] at the node
            pk[c][t] = rhs ? av : z[c * N + i] / g.dt - av;
        }
        double h, tvr = 0.0;
        for (int c = 0; c < 3; ++c) tvr = fma(tv[c], vr[c * N + i], tvr);
        if (rhs) {   // h(X, 0) + t . D_s (A f_ext) + t . D_s R[f_exp]
            h = g.cs[i] * 3.0 * E * ss3 + g.cc[i] * 3.0 * E * (sss3 + ss4) + al * E * ss4 + tdl + tdv;
            if (t == n - 1) {   // attached end: c (t . f_ext + 3 E X_ss . X_sss) + t . R[f_exp]
                double tfe = 0.0;
                for (int c = 0; c < 3; ++c) tfe = fma(tv[c], fe[c * N + i], tfe);
                cl_all[fl] = g.cc[i] * (tfe + 3.0 * E * ss3) + tvr;
            }
        } else {
            const double* zT = z + 3 * N + f0;
            double Ts = 0.0, Tss = 0.0;
            for (int k = 0; k < n; ++k) {
                Ts = fma(d1[k], zT[k], Ts);
                Tss = fma(d2[k], zT[k], Tss);
            }
            Ts *= s;
            Tss *= s * s;
            double k2 = 0.0;
            for (int c = 0; c < 3; ++c) k2 = fma(g.xss[c * N + i], g.xss[c * N + i], k2);
            ssf = -E * ss4 + k2 * zT[t];
            const double tf = 3.0 * E * ss3 + Ts, tf_s = 3.0 * E * (sss3 + ss4) + Tss;
            h = -(g.cs[i] * tf + g.cc[i] * tf_s - al * ssf + tdv);
            if (t == n - 1) cl_all[fl] = -(g.cc[i] * tf + tvr);   // attached end: -t . V[f]
        }
        hk[t] = h;
    }
    __syncthreads();
    if (!live) return;
    const int ek = end_kind(g, fi);
    const bool clamp = ek != 0;
    for (int r = t; r < 4 * n; r += 64) {
        double out = 0.0;
        int64_t dst;
        if (r < 3 * n) {
            const int c = r / n, j = r - c * n;
            dst = c * N + f0 + j;
            if (j < n - 4) {
                const double* p4 = g.P4 + j * n;
                for (int k = 0; k < n; ++k) out = fma(p4[k], pk[c][k], out);
            } else {
                const int b = j - (n - 4);                    // X_ss(L), X_sss(L), X_ss(0), X_sss(0)
                const int node = b < 2 ? 0 : n - 1;
                const double* u = z + c * N + f0;
                if (clamp && (b == 2 || (b == 3 && ek == 1))) {   // dX(0); clamped: D_s dX(0); rhs 0
                    if (!rhs) {
                        if (b == 2) {
                            out = u[n - 1];
                        } else {
                            const double* d1 = g.D1 + (n - 1) * n;
                            for (int k = 0; k < n; ++k) out = fma(d1[k], u[k] - u[0], out);
                            out *= s;
                        }
                    }
                } else {                                      // hinged b = 3: X_ss(0)
                    const bool d3 = b == 1 || (b == 3 && ek != 2);
                    const double* dm = (d3 ? g.D3 : g.D2) + node * n;
                    const double sc = d3 ? s * s * s : s * s;
                    for (int k = 0; k < n; ++k) out = fma(dm[k], u[k] - u[0], out);
                    out *= rhs ? -sc : sc;
                }
            }
        } else {
            const int j = r - 3 * n;
            dst = 3 * N + f0 + j;
            if (j < n - 2) {
                const double* p2 = g.P2 + j * n;
                for (int k = 0; k < n; ++k) out = fma(p2[k], hk[k], out);
            } else if (clamp && j == n - 1) {
                out = cl_all[fl];
            } else if (!rhs) {
                out = z[3 * N + f0 + (j == n - 2 ? 0 : n - 1)];
            }
        }
        w[dst] = out;
    }
}

// z = B_f^{-1} y on every fiber (inverse blocks column-major, m = 4 n).
__global__ __launch_bounds__(FB) void k_fs_precond(Geo g, const double* binv, const double* y,
                                                   double* z) {
    __shared__ double yl[GJ_MAX];
    const int n = g.n, m = 4 * n, f = blockIdx.x, t = threadIdx.x;
    const int64_t N = g.N, f0 = (int64_t)f * n;
    for (int c = t; c < m; c += FB) yl[c] = y[(c / n) * N + f0 + c % n];
    __syncthreads();
    const double* A = binv + (int64_t)f * m * m;
    for (int r = t; r < m; r += FB) {
        double acc = 0.0;
        for (int c = 0; c < m; ++c) acc = fma(A[(int64_t)c * m + r], yl[c], acc);
        z[(r / n) * N + f0 + r % n] = acc;
    }
}

// Block set-up, per fiber of a chunk: S = A + K_delta (3n x 3n: the node blocks A and,
// with the nonlocal term, the smooth pairs of K_delta), the self velocity of every
// unknown Vs = S F (3n x 4n), its smooth part Vm = (S - A) F, and the tension entries
// G[k][c] = h_k(unknown c) + t . D_s Vm[:, c] at node k (n x 4n).  Scratch per fiber:
// PREP_DOUBLES(n) doubles.
__host__ __device__ constexpr int64_t prep_doubles(int n) { return 37 * (int64_t)n * n; }

__global__ __launch_bounds__(FB) void k_fs_prep(Geo g, int f_begin, double* scratch) {
    const int n = g.n, m = 4 * n, n3 = 3 * n, f = f_begin + blockIdx.x, t = threadIdx.x;
    const int64_t N = g.N, f0 = (int64_t)f * n;
    double* S = scratch + (int64_t)blockIdx.x * prep_doubles(n);
    double* Vs = S + 9 * n * n;      // [3n][4n]
    double* Vm = Vs + 12 * n * n;    // [3n][4n]
    double* G = Vm + 12 * n * n;     // [n][4n]
    const double s = 2.0 / g.flen[f], d2 = g.delta * g.delta, E = g.E;
    // S[(a,i)][(b,l)], row-major 3n x 3n
    for (int e = t; e < n3 * n3; e += FB) {
        const int row = e / n3, col = e - row * n3;
        const int a = row / n, i = row - a * n, b = col / n, l = col - b * n;
        const int64_t gi = f0 + i, gl = f0 + l;
        const double id = a == b ? 1.0 : 0.0;
        double v = 0.0;
        if (l == i) {
            const double al = g.alpha[gi];
            v = al * id + (g.cc[gi] - al) * g.tan[a * N + gi] * g.tan[b * N + gi];
        } else if (g.nonlocal) {
            const double rx = g.X[gi] - g.X[gl], ry = g.X[N + gi] - g.X[N + gl],
                         rz = g.X[2 * N + gi] - g.X[2 * N + gl];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double ra = a == 0 ? rx : (a == 1 ? ry : rz);
            const double rb = b == 0 ? rx : (b == 1 ? ry : rz);
            v = g.pref * g.wq[gl] * (id + ra * rb / r2) / sqrt(r2 + d2);
        }
        S[e] = v;
    }
    __syncthreads();
    // Vs = S F: column (e, k) of F is -E s^4 D4[:, k] on component e; column T_k is
    // s D1[:, k] X_s(k) (X_s = s X_a) on every component.  Vm leaves out the node blocks.
    const double e4 = -E * s * s * s * s;
    for (int e = t; e < n3 * m; e += FB) {
        const int row = e / m, c = e - row * m, ri = row % n;
        const double* Sr = S + (int64_t)row * n3;
        double acc = 0.0, accm = 0.0;
        if (c < n3) {
            const int ce = c / n, k = c - ce * n;
            for (int l = 0; l < n; ++l) {
                const double q = Sr[ce * n + l] * g.D4[l * n + k];
                acc += q;
                if (l != ri) accm += q;
            }
            acc *= e4;
            accm *= e4;
        } else {
            const int k = c - n3;
            for (int b = 0; b < 3; ++b) {
                double q = 0.0, qm = 0.0;
                for (int l = 0; l < n; ++l) {
                    const double u = Sr[b * n + l] * g.D1[l * n + k];
                    q += u;
                    if (l != ri) qm += u;
                }
                acc = fma(q, g.Xa[b * N + f0 + k], acc);
                accm = fma(qm, g.Xa[b * N + f0 + k], accm);
            }
            acc *= s * s;
            accm *= s * s;
        }
        Vs[e] = acc;
        Vm[e] = accm;
    }
    __syncthreads();
    for (int e = t; e < n * m; e += FB) {
        const int k = e / m, c = e - k * m;
        const int64_t gk = f0 + k;
        double sm = 0.0;    // t . D_s Vm[:, c]
        for (int b = 0; b < 3; ++b) {
            double q = 0.0;
            for (int l = 0; l < n; ++l) q = fma(g.D1[k * n + l], Vm[(int64_t)(b * n + l) * m + c], q);
            sm = fma(q, g.tan[b * N + gk], sm);
        }
        sm *= s;
        double h;
        if (c < n3) {   // unit increment of component ce at node kc
            const int ce = c / n, kc = c - ce * n;
            const double x3 = s * s * s * g.D3[k * n + kc], x4 = s * s * s * s * g.D4[k * n + kc];
            const double xs2 = g.xss[ce * N + gk], xs3 = g.xsss[ce * N + gk];
            h = g.cs[gk] * 3.0 * E * xs2 * x3 + g.cc[gk] * 3.0 * E * (xs3 * x3 + xs2 * x4) +
                g.alpha[gk] * E * xs2 * x4;
        } else {        // unit tension at node kc
            const int kc = c - n3;
            double k2 = 0.0;
            for (int b = 0; b < 3; ++b) k2 = fma(g.xss[b * N + gk], g.xss[b * N + gk], k2);
            h = g.cs[gk] * s * g.D1[k * n + kc] + g.cc[gk] * s * s * g.D2[k * n + kc] -
                (k == kc ? g.alpha[gk] * k2 : 0.0);
        }
        G[e] = h + sm;
    }
}

// t . V of one unknown at the minus end (node n - 1) of fiber f: c (t . f) with
// t . f = 3 E X_ss . X_sss (unit increment) or T_s (unit tension), plus the smooth part
// t . Vm when Vm (the prepared smooth self velocity, 3n x 4n) is given.
__device__ double clamp_entry(const Geo& g, int f, int c, const double* Vm, double s) {
    const int n = g.n, m = 4 * n, n3 = 3 * n, p = n - 1;
    const int64_t N = g.N, i = (int64_t)f * n + p;
    double tf;
    if (c < n3) {
        const int ce = c / n, kc = c - ce * n;
        tf = 3.0 * g.E * g.xss[ce * N + i] * s * s * s * g.D3[p * n + kc];
    } else {
        tf = s * g.D1[p * n + (c - n3)];
    }
    double v = g.cc[i] * tf;
    if (Vm)
        for (int b = 0; b < 3; ++b) v = fma(g.tan[b * N + i], Vm[(int64_t)(b * n + p) * m + c], v);
    return v;
}

// Entries of the self block of each fiber of a chunk (rows as k_fs_rows, columns the
// unknowns dX_x, dX_y, dX_z, T of the fiber's nodes), inverted into binv.
__global__ __launch_bounds__(BLOCK_GJ) void k_fs_block(Geo g, int f_begin, const double* scratch,
                                                       double* binv) {
    __shared__ GjLds sh;
    const int n = g.n, m = 4 * n, n3 = 3 * n, f = f_begin + blockIdx.x, t = threadIdx.x;
    const double* Vs = scratch + (int64_t)blockIdx.x * prep_doubles(n) + 9 * n * n;
    const double* Vm = Vs + 12 * n * n;
    const double* G = Vs + 24 * n * n;
    const double s = 2.0 / g.flen[f];
    const int ek = end_kind(g, f);
    const bool clamp = ek != 0;
    const bool act = t < GJ_G * m;
    const int r = act ? t % m : 0, grp = act ? t / m : 0;
    double A[GJ_COLS];
#pragma unroll
    for (int jj = 0; jj < GJ_COLS; ++jj) {
        const int c = grp + GJ_G * jj;
        double v = 0.0;
        if (act && c < m) {
            const bool xcol = c < n3;
            const int ce = xcol ? c / n : 3, kc = xcol ? c - ce * n : c - n3;
            if (r < n3) {
                const int a = r / n, j = r - a * n;
                if (j < n - 4) {
                    const double* p4 = g.P4 + j * n;
                    for (int k = 0; k < n; ++k) v = fma(p4[k], -Vs[(int64_t)(a * n + k) * m + c], v);
                    if (xcol && ce == a) v += p4[kc] / g.dt;
                } else if (xcol && ce == a) {
                    const int b = j - (n - 4);
                    const int node = b < 2 ? 0 : n - 1;
                    if (clamp && b == 2)
                        v = kc == n - 1 ? 1.0 : 0.0;
                    else if (ek == 1 && b == 3)
                        v = s * g.D1[(n - 1) * n + kc];
                    else
                        v = (b == 1 || (b == 3 && ek != 2)) ? s * s * s * g.D3[node * n + kc]
                                                            : s * s * g.D2[node * n + kc];
                }
            } else {
                const int j = r - n3;
                if (j < n - 2) {
                    const double* p2 = g.P2 + j * n;
                    for (int k = 0; k < n; ++k) v = fma(p2[k], -G[(int64_t)k * m + c], v);
                } else if (clamp && j == n - 1) {
                    v = -clamp_entry(g, f, c, Vm, s);
                } else if (!xcol) {
                    v = kc == (j == n - 2 ? 0 : n - 1) ? 1.0 : 0.0;
                }
            }
        }
        A[jj] = v;
    }
    // row equilibration (as in k_fs_block64): the largest |entry| of each row over the
    // GJ_G column groups of its threads
    __shared__ double rmax[GJ_G][GJ_MAX], rscale[GJ_MAX];
    double mx = 0.0;
#pragma unroll
    for (int jj = 0; jj < GJ_COLS; ++jj) mx = fmax(mx, fabs(A[jj]));
    if (act) rmax[grp][r] = mx;
    __syncthreads();
    if (act) {
        double rm = 0.0;
        for (int q = 0; q < GJ_G; ++q) rm = fmax(rm, rmax[q][r]);
        const double d = rm > 0.0 && rm < INFINITY ? 1.0 / rm : 1.0;
#pragma unroll
        for (int jj = 0; jj < GJ_COLS; ++jj) A[jj] *= d;
        if (grp == 0) rscale[r] = d;
    }
    gj_invert(m, act, r, grp, A, sh, binv + (int64_t)f * m * m, rscale);
}

// Self blocks of fibers with at most 32 nodes (m = 4 n <= 128), one 256-thread workgroup
// per fiber (gj_invert64).  Without the nonlocal term the entries are formed here from
// the node data and the tables staged in LDS: the self velocity is node by node, so
// Vs[(a,k), c] = A_k F[(.,k), c].  With it they come from k_fs_prep's scratch.
constexpr int NB64 = 32;
template <bool LOCAL>
__global__ __launch_bounds__(GJ64_T) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_fs_block64(Geo g, int f_begin, const double* scratch,
                                                       double* binv) {
    // the tables of phase 1 and the elimination's LDS are never live together
    union Lds {
        struct {
            double d1[NB64 * NB64], d2[NB64 * NB64], d3[NB64 * NB64], d4[NB64 * NB64];
            double p4t[NB64 * NB64], p2t[NB64 * NB64];               // P4T[k][j], P2T[k][j]
            double nal[NB64], nbe[NB64], ncc[NB64], ncs[NB64], nk2[NB64];
            double nt[3][NB64], nxa[3][NB64], nxss[3][NB64], nxsss[3][NB64];
        } tb;
        Gj64Lds gj;
    };
    __shared__ Lds lds;
    Gj64Lds& sh = lds.gj;
    double *d1 = lds.tb.d1, *d2 = lds.tb.d2, *d3 = lds.tb.d3, *d4 = lds.tb.d4, *p4t = lds.tb.p4t,
           *p2t = lds.tb.p2t, *nal = lds.tb.nal, *nbe = lds.tb.nbe, *ncc = lds.tb.ncc, *ncs = lds.tb.ncs,
           *nk2 = lds.tb.nk2;
    double(*nt)[NB64] = lds.tb.nt;
    double(*nxa)[NB64] = lds.tb.nxa;
    double(*nxss)[NB64] = lds.tb.nxss;
    double(*nxsss)[NB64] = lds.tb.nxsss;
    const int n = g.n, m = 4 * n, n3 = 3 * n, t = threadIdx.x;
    const int fl = blockIdx.x, f = f_begin + fl;
    const int64_t N = g.N, f0 = (int64_t)f * n;
    const double s = 2.0 / g.flen[f], E = g.E;
    for (int e = t; e < n * n; e += GJ64_T) {
        d1[e] = g.D1[e];
        d2[e] = g.D2[e];
        d3[e] = g.D3[e];
        d4[e] = g.D4[e];
        const int k = e / n, j = e - k * n;              // transposed resampling tables
        if (j < n - 4) p4t[e] = g.P4[j * n + k];
        if (j < n - 2) p2t[e] = g.P2[j * n + k];
    }
    if (t < n) {
        const int64_t i = f0 + t;
        nal[t] = g.alpha[i];
        ncc[t] = g.cc[i];
        nbe[t] = g.cc[i] - g.alpha[i];
        ncs[t] = g.cs[i];
        double k2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            nt[c][t] = g.tan[c * N + i];
            nxa[c][t] = g.Xa[c * N + i];
            nxss[c][t] = g.xss[c * N + i];
            nxsss[c][t] = g.xsss[c * N + i];
            k2 = fma(g.xss[c * N + i], g.xss[c * N + i], k2);
        }
        nk2[t] = k2;
    }
    __syncthreads();
    // (entries formed in place: no scratch, and the launch may cover more fibers than a chunk)
    const double* Vs = LOCAL ? nullptr : scratch + (int64_t)fl * prep_doubles(n) + 9 * n * n;
    const double* G = LOCAL ? nullptr : Vs + 24 * n * n;
    const double e4 = -E * s * s * s * s, s2 = s * s, s3 = s2 * s, s4 = s2 * s2;
    const int ek = end_kind(g, f);
    const bool clamp = ek != 0;
    double* Bf = binv + (int64_t)f * m * m;
    // phase 1: the block, column-major, into its own inverse slot.
    if constexpr (LOCAL) {
        // Interior rows, as sums over the fiber's nodes k of L[k][j] R(k, c): the
        // resampling table L (P4 for the position rows of component a, P2 for the
        // tension rows) does not depend on the column, so a thread takes one column c of
        // one row block, forms R(k, c) once per node and adds it to all the block's rows,
        // whose L values every thread of the wave reads at the same LDS address.
        for (int task = t; task < 4 * m; task += GJ64_T) {
            const int rb = task / m, c = task - rb * m;   // rb: position component 0..2, or 3 (tension)
            const bool xcol = c < n3;
            const int ce = xcol ? c / n : 3, kc = xcol ? c - ce * n : c - n3;
            const int nr = rb < 3 ? n - 4 : n - 2;
            const double* L = rb < 3 ? p4t : p2t;
            double acc[NB64 - 2];
#pragma unroll
            for (int jj = 0; jj < NB64 - 2; ++jj) acc[jj] = 0.0;
            for (int k = 0; k < n; ++k) {
                double R;
                if (rb < 3) {
                    const int a = rb;
                    if (xcol) {
                        const double Ake = (a == ce ? nal[k] : 0.0) + nbe[k] * nt[a][k] * nt[ce][k];
                        R = Ake * d4[k * n + kc];
                    } else {
                        const double xa0 = nxa[0][kc], xa1 = nxa[1][kc], xa2 = nxa[2][kc];
                        const double xaa = a == 0 ? xa0 : (a == 1 ? xa1 : xa2);
                        const double tx = nt[0][k] * xa0 + nt[1][k] * xa1 + nt[2][k] * xa2;
                        R = d1[k * n + kc] * (nal[k] * xaa + nbe[k] * nt[a][k] * tx);
                    }
                } else if (xcol) {
                    const double x3 = s3 * d3[k * n + kc], x4 = s4 * d4[k * n + kc];
                    const double xs2 = nxss[ce][k], xs3 = nxsss[ce][k];
                    R = ncs[k] * 3.0 * E * xs2 * x3 + ncc[k] * 3.0 * E * (xs3 * x3 + xs2 * x4) +
                        nal[k] * E * xs2 * x4;
                } else {
                    R = ncs[k] * s * d1[k * n + kc] + ncc[k] * s2 * d2[k * n + kc] -
                        (k == kc ? nal[k] * nk2[k] : 0.0);
                }
                const double* Lk = L + k * n;
#pragma unroll
                for (int jj = 0; jj < NB64 - 2; ++jj)
                    if (jj < nr) acc[jj] = fma(Lk[jj], R, acc[jj]);
            }
            const double sc = rb < 3 ? (xcol ? -e4 : -s2) : -1.0;
#pragma unroll
            for (int jj = 0; jj < NB64 - 2; ++jj)
                if (jj < nr) {
                    double v = acc[jj] * sc;
                    if (rb < 3 && xcol && ce == rb) v += p4t[kc * n + jj] / g.dt;
                    Bf[(int64_t)c * m + (rb < 3 ? rb * n + jj : n3 + jj)] = v;
                }
        }
        // the boundary rows: the last four position rows of each component, the last two
        // tension rows
        const int xb0 = n > 4 ? n - 4 : 0, tb0 = n > 2 ? n - 2 : 0;
        const int nbx = n - xb0, nbr = 3 * nbx + (n - tb0);
        for (int e = t; e < nbr * m; e += GJ64_T) {
            const int c = e / nbr, q = e - c * nbr;
            const bool xcol = c < n3;
            const int ce = xcol ? c / n : 3, kc = xcol ? c - ce * n : c - n3;
            double v = 0.0;
            int r;
            if (q < 3 * nbx) {
                const int a = q / nbx, j = xb0 + (q - a * nbx);
                r = a * n + j;
                if (xcol && ce == a) {
                    const int b = j - (n - 4);
                    const int node = b < 2 ? 0 : n - 1;
                    if (clamp && b == 2)
                        v = kc == n - 1 ? 1.0 : 0.0;
                    else if (ek == 1 && b == 3)
                        v = s * d1[(n - 1) * n + kc];
                    else
                        v = (b == 1 || (b == 3 && ek != 2)) ? s3 * d3[node * n + kc] : s2 * d2[node * n + kc];
                }
            } else {
                const int j = tb0 + (q - 3 * nbx);
                r = n3 + j;
                if (clamp && j == n - 1)
                    v = -clamp_entry(g, f, c, nullptr, s);
                else if (!xcol)
                    v = kc == (j == n - 2 ? 0 : n - 1) ? 1.0 : 0.0;
            }
            Bf[(int64_t)c * m + r] = v;
        }
    } else {
    // (from the prepared products: consecutive threads
    // take consecutive rows of one column)
    for (int e = t; e < m * m; e += GJ64_T) {
        const int c = e / m, r = e - c * m;
        double v = 0.0;
        const bool xcol = c < n3;
        const int ce = xcol ? c / n : 3, kc = xcol ? c - ce * n : c - n3;
        if (r < n3) {
            const int a = r / n, j = r - a * n;
            if (j < n - 4) {
                if (LOCAL) {
                    if (xcol) {
                        for (int k = 0; k < n; ++k) {
                            const double Ake = (a == ce ? nal[k] : 0.0) + nbe[k] * nt[a][k] * nt[ce][k];
                            v = fma(p4t[k * n + j] * Ake, d4[k * n + kc], v);
                        }
                        v *= -e4;
                    } else {
                        const double xa0 = nxa[0][kc], xa1 = nxa[1][kc], xa2 = nxa[2][kc];
                        const double xaa = a == 0 ? xa0 : (a == 1 ? xa1 : xa2);
                        for (int k = 0; k < n; ++k) {
                            const double tx = nt[0][k] * xa0 + nt[1][k] * xa1 + nt[2][k] * xa2;
                            const double ax = nal[k] * xaa + nbe[k] * nt[a][k] * tx;
                            v = fma(p4t[k * n + j] * d1[k * n + kc], ax, v);
                        }
                        v *= -s2;
                    }
                } else {
                    for (int k = 0; k < n; ++k) v = fma(p4t[k * n + j], -Vs[(int64_t)(a * n + k) * m + c], v);
                }
                if (xcol && ce == a) v += p4t[kc * n + j] / g.dt;
            } else if (xcol && ce == a) {
                const int b = j - (n - 4);
                const int node = b < 2 ? 0 : n - 1;
                if (clamp && b == 2)
                    v = kc == n - 1 ? 1.0 : 0.0;
                else if (ek == 1 && b == 3)
                    v = s * d1[(n - 1) * n + kc];
                else
                    v = (b == 1 || (b == 3 && ek != 2)) ? s3 * d3[node * n + kc] : s2 * d2[node * n + kc];
            }
        } else {
            const int j = r - n3;
            if (j < n - 2) {
                if (LOCAL) {
                    if (xcol) {
                        for (int k = 0; k < n; ++k) {
                            const double x3 = s3 * d3[k * n + kc], x4 = s4 * d4[k * n + kc];
                            const double xs2 = nxss[ce][k], xs3 = nxsss[ce][k];
                            const double h = ncs[k] * 3.0 * E * xs2 * x3 +
                                             ncc[k] * 3.0 * E * (xs3 * x3 + xs2 * x4) + nal[k] * E * xs2 * x4;
                            v = fma(p2t[k * n + j], h, v);
                        }
                    } else {
                        for (int k = 0; k < n; ++k) {
                            const double h = ncs[k] * s * d1[k * n + kc] + ncc[k] * s2 * d2[k * n + kc] -
                                             (k == kc ? nal[k] * nk2[k] : 0.0);
                            v = fma(p2t[k * n + j], h, v);
                        }
                    }
                    v = -v;
                } else {
                    for (int k = 0; k < n; ++k) v = fma(p2t[k * n + j], -G[(int64_t)k * m + c], v);
                }
            } else if (clamp && j == n - 1) {
                v = -clamp_entry(g, f, c, LOCAL ? nullptr : Vs + 12 * n * n, s);
            } else if (!xcol) {
                v = kc == (j == n - 2 ? 0 : n - 1) ? 1.0 : 0.0;
            }
        }
        Bf[e] = v;
    }
    }
    __threadfence_block();
    __syncthreads();
    // phase 2: each thread's row segment into registers, then Gauss-Jordan in place
    const bool act = t < 2 * m;
    const int r = act ? t % m : 0, grp = act ? t / m : 0;
    double A[64], mx = 0.0;
#pragma unroll
    for (int jj = 0; jj < 64; ++jj) {
        const int c = grp * 64 + jj;
        A[jj] = (act && c < m) ? Bf[(int64_t)c * m + r] : 0.0;
        mx = fmax(mx, fabs(A[jj]));
    }
    // row equilibration: the rows span many orders of magnitude (E M D_s^4 against the
    // boundary and tension rows), which Gauss-Jordan in FP64 does not survive unscaled
    __shared__ double rmax[2][GJ64_MAX], rscale[GJ64_MAX];
    if (act) rmax[grp][r] = mx;
    __syncthreads();   // (also: every load done before any thread writes the inverse)
    if (act) {
        const double rm = fmax(rmax[0][r], rmax[1][r]);
        const double d = rm > 0.0 && rm < INFINITY ? 1.0 / rm : 1.0;
#pragma unroll
        for (int jj = 0; jj < 64; ++jj) A[jj] *= d;
        if (grp == 0) rscale[r] = d;
    }
    gj_invert64(m, act, r, grp, A, sh, Bf, rscale);
}

__global__ __launch_bounds__(EB) void k_fs_finish(int64_t N, const double* X, const double* x,
                                                  double* xyz_out, double* T_out) {
    const int64_t i = (int64_t)blockIdx.x * EB + threadIdx.x;
    if (i >= N) return;
    for (int c = 0; c < 3; ++c) xyz_out[c * N + i] = X[c * N + i] + x[c * N + i];
    T_out[i] = x[3 * N + i];
}

inline unsigned grid_e(int64_t n) { return (unsigned)((n + EB - 1) / EB); }

// Device memory of the step, kept per (device, stream) between calls: a call is
// synchronous, so the next call on the same stream may reuse it.  tab_n records the
// nodes per fiber whose tables sit at the start of the buffer.
struct StepBuf {
    int dev = 0;
    hipStream_t st = nullptr;
    void* p = nullptr;
    size_t bytes = 0;
    int tab_n = 0;
    // the block set-up runs on a side stream, beside the right-hand side on st
    hipStream_t side = nullptr;
    hipEvent_t ev_geom = nullptr, ev_blk = nullptr;
};
static std::mutex g_step_mu;
static std::vector<StepBuf> g_step_bufs;

static int step_buffer(hipStream_t st, size_t bytes, StepBuf* out) {
    int dev = 0;
    STOKES_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_step_mu);
    for (auto& b : g_step_bufs)
        if (b.dev == dev && b.st == st) {
            if (b.bytes < bytes) {
                STOKES_HIP(hipFree(b.p));
                b.p = nullptr;
                b.bytes = 0;
                b.tab_n = 0;
                STOKES_HIP(hipMalloc(&b.p, bytes));
                b.bytes = bytes;
            }
            *out = b;
            return STOKES_OK;
        }
    StepBuf b;
    b.dev = dev;
    b.st = st;
    STOKES_HIP(hipStreamCreateWithFlags(&b.side, hipStreamNonBlocking));   // (default priority)
    STOKES_HIP(hipEventCreateWithFlags(&b.ev_geom, hipEventDisableTiming));
    STOKES_HIP(hipEventCreateWithFlags(&b.ev_blk, hipEventDisableTiming));
    STOKES_HIP(hipMalloc(&b.p, bytes));
    b.bytes = bytes;
    g_step_bufs.push_back(b);
    *out = b;
    return STOKES_OK;
}

// Joins the side stream into st: everything launched on sd so far completes before
// later work on st.  join() at the join point; the destructor joins on early returns
// too, so that a later call on st never overlaps this call's side work.
struct SideJoin {
    hipStream_t st, sd;
    hipEvent_t ev;
    bool open = true;
    int join() {
        open = false;
        STOKES_HIP(hipEventRecord(ev, sd));
        STOKES_HIP(hipStreamWaitEvent(st, ev, 0));
        return STOKES_OK;
    }
    ~SideJoin() {
        if (open) {
            (void)hipEventRecord(ev, sd);
            (void)hipStreamWaitEvent(st, ev, 0);
        }
    }
};

static void step_tables_loaded(hipStream_t st, int n) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_step_mu);
    for (auto& b : g_step_bufs)
        if (b.dev == dev && b.st == st) b.tab_n = n;
}

}  // namespace fs

// Frees the step buffers (called by stokes_release_workspace after a device sync).
void fiberstep_release() {
    std::lock_guard<std::mutex> lk(fs::g_step_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& b : fs::g_step_bufs) {
        (void)hipSetDevice(b.dev);
        (void)hipDeviceSynchronize();
        if (b.p) (void)hipFree(b.p);
        if (b.ev_geom) (void)hipEventDestroy(b.ev_geom);
        if (b.ev_blk) (void)hipEventDestroy(b.ev_blk);
        if (b.side) (void)hipStreamDestroy(b.side);
    }
    (void)hipSetDevice(cur);
    fs::g_step_bufs.clear();
}

}  // namespace stokes

using namespace stokes;
using namespace stokes::fs;

extern "C" int stokes_fiber_step(int32_t n_fib, int32_t nodes_per_fib, const double* xyz,
                                 const double* fiber_len, const double* f_ext,
                                 const int32_t* clamp_minus, double eps, double E,
                                 double dt, double mu, double delta, double near_r, int32_t iters,
                                 double tol, uint32_t flags, double* xyz_out, double* T_out,
                                 double* resid_out, int32_t* iters_out, const stokes_far* far,
                                 void* stream) {
    const char* who = "stokes_fiber_step: ";
    const int n = nodes_per_fib;
    if (int rc = check_far(far, "stokes_fiber_step")) return rc;
    if (n_fib < 0 || n < 6 || n > MAX_NPF)
        return fail(STOKES_E_INVAL, std::string(who) + "need n_fib >= 0 and 6 <= nodes_per_fib <= " +
                                        std::to_string(MAX_NPF));
    if (!(mu > 0.0) || !std::isfinite(mu)) return fail(STOKES_E_INVAL, std::string(who) + "mu must be > 0");
    if (!(eps > 0.0 && eps < 0.5)) return fail(STOKES_E_INVAL, std::string(who) + "eps must be in (0, 0.5)");
    if (!(E >= 0.0) || !std::isfinite(E)) return fail(STOKES_E_INVAL, std::string(who) + "E must be finite and >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(STOKES_E_INVAL, std::string(who) + "dt must be finite and > 0");
    if (!(tol >= 0.0)) return fail(STOKES_E_INVAL, std::string(who) + "tol must be >= 0");
    if (iters < 1 || iters > STOKES_MAX_ITERS)
        return fail(STOKES_E_INVAL, std::string(who) + "iters must be in 1..STOKES_MAX_ITERS");
    const bool nonlocal = flags & STOKES_NONLOCAL;
    if (nonlocal && (!(delta > 0.0) || !std::isfinite(delta)))
        return fail(STOKES_E_INVAL, std::string(who) + "delta must be finite and > 0 with STOKES_NONLOCAL");
    const uint32_t known = STOKES_PREC_MIXED | STOKES_NO_DOUBLET | STOKES_NONLOCAL;
    if (flags & ~known) return fail(STOKES_E_INVAL, std::string(who) + "unsupported flag");
    const int64_t N = (int64_t)n_fib * n;
    if (N >= (int64_t)1 << 28) return fail(STOKES_E_INVAL, std::string(who) + "too many nodes");
    if (resid_out) *resid_out = 0.0;
    if (iters_out) *iters_out = 0;
    if (N == 0) return STOKES_OK;
    Range range("stokes_fiber_step");
    if (!xyz || !fiber_len || !f_ext || !xyz_out || !T_out)
        return fail(STOKES_E_INVAL, std::string(who) + "null pointer");
    if (xyz_out == xyz || xyz_out == f_ext)
        return fail(STOKES_E_INVAL, std::string(who) + "xyz_out must not alias an input");
    hipStream_t st = static_cast<hipStream_t>(stream);

    const int m = 4 * n;
    const int64_t n_vec = (4 * N + 2) / 3, nv3 = 3 * n_vec;
    const int chunk = std::min(n_fib, PREP_CHUNK);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_tab = take((size_t)(4 * n * n + (n - 4) * n + (n - 2) * n) * 8),
                 o_Xa = take(3 * N * 8), o_tan = take(3 * N * 8), o_wq = take(N * 8), o_sarc = take(N * 8),
                 o_xss = take(3 * N * 8), o_xsss = take(3 * N * 8), o_al = take(N * 8), o_cc = take(N * 8),
                 o_cs = take(N * 8),
                 o_fib = take(N * 4), o_f = take(3 * N * 8), o_v = take(3 * N * 8), o_rhs = take(nv3 * 8),
                 o_binv = take((size_t)n_fib * m * m * 8), o_prep = take((size_t)chunk * prep_doubles(n) * 8),
                 o_slot = take(vector_plan_bytes(n_vec, iters));
    StepBuf buf;
    int rc0 = step_buffer(st, off, &buf);
    if (rc0) return rc0;
    char* base = static_cast<char*>(buf.p);
    auto at = [&](size_t o) { return reinterpret_cast<double*>(base + o); };
    double* dtab = at(o_tab);
    if (buf.tab_n != n) {
        const cheb::Tables tab = cheb::build(n);
        std::vector<double> h;
        h.reserve(4 * n * n + 2 * n * n);
        for (const auto* v : {&tab.D1, &tab.D2, &tab.D3, &tab.D4, &tab.P4, &tab.P2})
            h.insert(h.end(), v->begin(), v->end());
        STOKES_HIP(hipMemcpyAsync(dtab, h.data(), h.size() * 8, hipMemcpyHostToDevice, st));
        STOKES_HIP(hipStreamSynchronize(st));   // h is a pageable host buffer
        step_tables_loaded(st, n);
    }
    double *Xa = at(o_Xa), *tan = at(o_tan), *wq = at(o_wq), *sarc = at(o_sarc), *fbuf = at(o_f),
           *vbuf = at(o_v), *rhs = at(o_rhs), *binv = at(o_binv), *prep = at(o_prep), *xss = at(o_xss),
           *xsss = at(o_xsss), *alpha = at(o_al), *ccoef = at(o_cc), *cs = at(o_cs);
    int32_t* fib = reinterpret_cast<int32_t*>(base + o_fib);
    void* slot = base + o_slot;

    Geo g{};
    g.N = N;
    g.n = n;
    g.nf = n_fib;
    g.X = xyz;
    g.flen = fiber_len;
    g.clamp = clamp_minus;
    g.Xa = Xa;
    g.tan = tan;
    g.wq = wq;
    g.sarc = sarc;
    g.xss = xss;
    g.xsss = xsss;
    g.alpha = alpha;
    g.cc = ccoef;
    g.cs = cs;
    g.D1 = dtab;
    g.D2 = dtab + n * n;
    g.D3 = dtab + 2 * n * n;
    g.D4 = dtab + 3 * n * n;
    g.P4 = dtab + 4 * n * n;
    g.P2 = g.P4 + (n - 4) * n;
    g.E = E;
    g.dt = dt;
    g.mu = mu;
    g.kappa = -log(eps * eps * M_E);
    g.pref = 1.0 / (8.0 * M_PI * mu);
    g.delta = nonlocal ? delta : 1.0;
    g.nonlocal = nonlocal;

    const uint32_t sumflags = (flags & (STOKES_PREC_MIXED | STOKES_NO_DOUBLET)) | STOKES_EXCL_SAME_FIBER |
                              STOKES_ACCUMULATE;
    // the other fibers' flow through a treecode plan of this step's nodes, if asked for
    FarPlan fp;
    if (far) {
        if (int rc = fp.make(N, xyz, *far, st)) return rc;
    }
    // vr = R[f]: the smooth part of K_delta f, then the other fibers' flow added in
    auto smooth_velocity = [&](const double* f, double* vr) -> int {
        hipLaunchKernelGGL(k_fs_smooth, dim3(grid_e(N)), dim3(EB), 0, st, g, f, vr);
        STOKES_HIP(hipGetLastError());
        if (far)
            return stokes_tree_sl_eval(fp.t, f, wq, fib, n_fib, fiber_len, mu, eps, near_r, sumflags, vr, st);
        return stokes_sl_eval(N, xyz, f, wq, fib, n_fib, fiber_len, N, xyz, nullptr, fib, mu, eps, near_r,
                              sumflags, vr, st, nullptr);
    };

    hipLaunchKernelGGL(k_fs_geom, dim3(grid_e(N)), dim3(EB), 0, st, g, Xa, tan, wq, sarc, fib, xss, xsss,
                       alpha, ccoef);
    hipLaunchKernelGGL(k_fs_geom2, dim3(grid_e(N)), dim3(EB), 0, st, g, cs);
    STOKES_HIP(hipGetLastError());
    // the preconditioner's blocks on the side stream, beside the right-hand side (both
    // need only the geometry; the blocks are latency-bound, the right-hand side's pair
    // sums are not), joined before the first GMRES iteration
    const hipStream_t sd = buf.side;
    STOKES_HIP(hipEventRecord(buf.ev_geom, st));
    STOKES_HIP(hipStreamWaitEvent(sd, buf.ev_geom, 0));
    SideJoin sj{st, sd, buf.ev_blk};
    if (n <= NB64 && !nonlocal) {   // entries formed in place: no scratch, one launch
        hipLaunchKernelGGL(k_fs_block64<true>, dim3(n_fib), dim3(GJ64_T), 0, sd, g, 0, (const double*)prep, binv);
        STOKES_HIP(hipGetLastError());
    } else
    for (int f0 = 0; f0 < n_fib; f0 += chunk) {
        const int nb = std::min(chunk, n_fib - f0);
        {
            hipLaunchKernelGGL(k_fs_prep, dim3(nb), dim3(FB), 0, sd, g, f0, prep);
            if (n <= NB64)
                hipLaunchKernelGGL(k_fs_block64<false>, dim3(nb), dim3(GJ64_T), 0, sd, g, f0,
                                   (const double*)prep, binv);
            else
                hipLaunchKernelGGL(k_fs_block, dim3(nb), dim3(BLOCK_GJ), 0, sd, g, f0, (const double*)prep, binv);
        }
        STOKES_HIP(hipGetLastError());
    }
    // right-hand side: the rows of f_exp = f_ext - E s^4 D4 X with the current nodes
    STOKES_HIP(hipMemsetAsync(rhs, 0, nv3 * 8, st));
    hipLaunchKernelGGL(k_fs_force, dim3(grid_e(N)), dim3(EB), 0, st, g, xyz, (const double*)nullptr, f_ext,
                       fbuf);
    STOKES_HIP(hipGetLastError());
    int rc = smooth_velocity(fbuf, vbuf);
    const unsigned rows_grid = (unsigned)((n_fib + ROWS_FPB - 1) / ROWS_FPB);
    if (!rc)
        hipLaunchKernelGGL(k_fs_rows, dim3(rows_grid), dim3(64 * ROWS_FPB), 0, st, g, xyz, (const double*)fbuf,
                           (const double*)vbuf, f_ext, true, rhs);
    if (int jr = sj.join()) return jr;
    if (rc) return rc;
    STOKES_HIP(hipGetLastError());

    // w = A B^{-1} v: z = B^{-1} v, f = F z, vr = R[f], w = rows(z, f, vr)
    auto apply = [&](const double* v, double* z, double* w) -> int {
        hipLaunchKernelGGL(k_fs_precond, dim3(n_fib), dim3(FB), 0, st, g, (const double*)binv, v, z);
        hipLaunchKernelGGL(k_fs_force, dim3(grid_e(N)), dim3(EB), 0, st, g, (const double*)z,
                           (const double*)(z + 3 * N), (const double*)nullptr, fbuf);
        STOKES_HIP(hipGetLastError());
        const int r2 = smooth_velocity(fbuf, vbuf);
        if (r2) return r2;
        hipLaunchKernelGGL(k_fs_rows, dim3(rows_grid), dim3(64 * ROWS_FPB), 0, st, g, (const double*)z,
                           (const double*)fbuf, (const double*)vbuf, (const double*)nullptr, false, w);
        STOKES_HIP(hipGetLastError());
        return STOKES_OK;
    };

    Batch b;
    if ((rc = b.init(st, false, true, false))) return rc;
    if ((rc = b.attach_vector(0, slot, n_vec, iters, rhs))) return rc;
    {
        SlotDesc& d = b.desc(0);
        if (nv3 > 4 * N) STOKES_HIP(hipMemsetAsync(d.w + 4 * N, 0, (nv3 - 4 * N) * 8, st));
    }
    const std::vector<int> one{0};
    if ((rc = b.start_vector(one))) return rc;
    int done = 0;
    const double beta = b.status(0)[1];
    double resid = b.status(0)[2];
    if (b.status(0)[3] == 0.0 && beta > 0.0) {
        for (int j = 0; j < iters; ++j) {
            SlotDesc& d = b.desc(0);
            d.j = j;
            if ((rc = apply(d.V + (int64_t)j * nv3, d.z, d.w))) return rc;
            if ((rc = b.step_ortho(one))) return rc;
            done = j + 1;
            resid = b.status(0)[2];
            if (b.status(0)[3] != 0.0) break;          // exact breakdown
            if (resid <= tol * beta) break;
        }
    }
    b.desc(0).j = done;
    if ((rc = b.finalize_vector(one))) return rc;
    SlotDesc& d = b.desc(0);
    hipLaunchKernelGGL(k_fs_precond, dim3(n_fib), dim3(FB), 0, st, g, (const double*)binv,
                       (const double*)d.w, d.x);
    hipLaunchKernelGGL(k_fs_finish, dim3(grid_e(N)), dim3(EB), 0, st, N, xyz, (const double*)d.x, xyz_out,
                       T_out);
    STOKES_HIP(hipGetLastError());
    STOKES_HIP(hipStreamSynchronize(st));
    if (resid_out) *resid_out = resid;
    if (iters_out) *iters_out = done;
    return STOKES_OK;
}
