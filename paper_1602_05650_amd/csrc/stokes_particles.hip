// Rigid particles in a confining periphery: the second-kind boundary integral
// mobility problem (eq. main-cortex-density with the rank completion N of
// eq. main-cortex-vel; eq. main-nsb-second-kind with the constraints
// eq. main-nsb-rgbt and eq. main-nsb-rgbr), Nystrom-discretised on the given
// surface quadratures, solved by right-preconditioned GMRES with the diagonal
// Jacobi preconditioner of eq. prec.
//
// With K the double-layer sum of stokes_dl_eval (outward normals; -q inside,
// -q/2 on the surface, 0 outside), the paper's double layer with the normal into
// the fluid is +K on the periphery and -K on a particle, and the equations are
//
//   x on Gamma_0:  -q0/2 + K0_PV[q0] + n(x) int n.q0 dS - sum_p K_p[q_p]   = b(x)
//   x on P_p:      -q_p/2 + K0[q0] - sum_p' K_p'[q_p'] (own term PV)
//                  - U_p - Omega_p x (x - X_p)                             = b(x)
//   (1/|P_p|) int q_p dS - U_p = 0,  (1/|P_p|) int (y - X_p) x q_p dS - Omega_p = 0
//
// b(x) = -sum_p [G(x - X_p) F_p + R(x - X_p) L_p]  (eq. oseen, eq. rotlet).
// Unknowns: three planes of n_tot = M_s + 2 n_p entries,
// [q on the M_s surface points (periphery first) | U_1..U_np | Omega_1..Omega_np].
#include <math.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "solver_batch.hpp"

namespace stokes {
namespace pt {

constexpr int PB = 256;
constexpr double PI = 3.14159265358979323846;

// Surfaces: index 0 is the periphery (possibly empty), 1 + p is particle p.  Each
// surface's points are a contiguous SoA block (three planes of its size) in the
// block arrays; point i of the concatenated surface list belongs to surface sid[i]
// and sits at local index i - sstart[sid[i]].
struct Surfaces {
    const double* xyz;      // blocks: surface s at 3 * sstart[s], planes of ssize[s]
    const double* nrm;
    const double* w;        // [M_s], concatenated
    const int32_t* sid;     // [M_s]
    const int64_t* sstart;  // [n_surf]
    const int64_t* ssize;   // [n_surf]
};

__device__ __forceinline__ const double* block(const double* a, const Surfaces& S, int s) {
    return a + 3 * S.sstart[s];
}

// b = -sum_p [G(x - X_p) F_p + R(x - X_p) L_p] on the surface points, 0 on the U, Omega rows.
__global__ __launch_bounds__(PB) void k_pt_rhs(int64_t ms, int64_t ntot, const double* T, int32_t np,
                                               const double* X, const double* F, const double* L,
                                               double mu, double* b) {
    const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
    if (i >= ntot) return;
    double u0 = 0.0, u1 = 0.0, u2 = 0.0;
    if (i < ms) {
        const double x = T[i], y = T[ms + i], z = T[2 * ms + i];
        for (int p = 0; p < np; ++p) {
            const double rx = x - X[p], ry = y - X[np + p], rz = z - X[2 * np + p];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double rn = sqrt(r2);
            const double ri = 1.0 / rn, ri3 = ri / r2;
            const double fx = F[p], fy = F[np + p], fz = F[2 * np + p];
            const double lx = L[p], ly = L[np + p], lz = L[2 * np + p];
            const double rf = (rx * fx + ry * fy + rz * fz) * ri3;
            u0 += fx * ri + rx * rf + (ly * rz - lz * ry) * ri3;
            u1 += fy * ri + ry * rf + (lz * rx - lx * rz) * ri3;
            u2 += fz * ri + rz * rf + (lx * ry - ly * rx) * ri3;
        }
        const double c = -1.0 / (8.0 * PI * mu);
        u0 *= c;
        u1 *= c;
        u2 *= c;
    }
    b[i] = u0;
    b[ntot + i] = u1;
    b[2 * ntot + i] = u2;
}

// Diagonal of the self-interaction blocks: on the periphery -1 - sum_s w_s K_cc + w n_c^2,
// on a particle sum_s w_s K_cc over its own points (s != i), -1 on the U, Omega rows.
// One wave per row: lane l sums the points k = l, l + 64, ... of the row's surface, and
// the 64 partial sums are combined by a fixed butterfly (the periphery's rows each
// cover all its points; a thread per row would leave the chip nearly idle).
__global__ __launch_bounds__(64) void k_pt_diag(Surfaces S, int64_t ms, int64_t ntot, double* diag) {
    const int64_t i = blockIdx.x;
    const int l = threadIdx.x;
    double d0 = -1.0, d1 = -1.0, d2 = -1.0;
    if (i < ms) {
        const int s = S.sid[i];
        const int64_t n = S.ssize[s], li = i - S.sstart[s];
        const double* y = block(S.xyz, S, s);
        const double* nn = block(S.nrm, S, s);
        const double* w = S.w + S.sstart[s];
        const double xi = y[li], yi = y[n + li], zi = y[2 * n + li];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t k = l; k < n; k += 64) {
            if (k == li) continue;
            const double dx = xi - y[k], dy = yi - y[n + k], dz = zi - y[2 * n + k];
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double dn = dx * nn[k] + dy * nn[n + k] + dz * nn[2 * n + k];
            const double c = 3.0 / (4.0 * PI) * w[k] * dn / (r2 * r2 * sqrt(r2));
            a0 += c * dx * dx;
            a1 += c * dy * dy;
            a2 += c * dz * dz;
        }
        for (int o = 32; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o, 64);
            a1 += __shfl_xor(a1, o, 64);
            a2 += __shfl_xor(a2, o, 64);
        }
        if (s == 0) {
            const double wi = w[li];
            d0 = -1.0 - a0 + wi * nn[li] * nn[li];
            d1 = -1.0 - a1 + wi * nn[n + li] * nn[n + li];
            d2 = -1.0 - a2 + wi * nn[2 * n + li] * nn[2 * n + li];
        } else {
            d0 = a0;
            d1 = a1;
            d2 = a2;
        }
    }
    if (l == 0) {
        diag[i] = d0;
        diag[ntot + i] = d1;
        diag[2 * ntot + i] = d2;
    }
}

// The solve's geometry from the caller's arrays, one thread per surface point i: points
// T and normals NS as planes of M_s (periphery first, then the particles in order), the
// per-surface blocks bx, bn of Surfaces, the weights bw, surface ids sid (0 the
// periphery, 1 + p particle p) and self indices (i).  po = part_offset (strictly
// increasing: every particle has at least four points).
__global__ __launch_bounds__(PB) void k_pt_geometry(int64_t m0, const double* y0, const double* n0,
                                                    const double* w0, int64_t mp, const double* yp,
                                                    const double* np_, const double* wp, int32_t n_part,
                                                    const int64_t* po, double* T, double* NS, double* bx,
                                                    double* bn, double* bw, int32_t* sid, int64_t* self) {
    const int64_t ms = m0 + mp;
    const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
    if (i >= ms) return;
    const double *y, *nn;
    int64_t ns, k, li, n, start;
    int s;
    double w;
    if (i < m0) {
        s = 0;
        y = y0;
        nn = n0;
        ns = m0;
        k = li = i;
        n = m0;
        start = 0;
        w = w0[i];
    } else {
        k = i - m0;
        int lo = 0, hi = n_part;   // po[lo] <= k < po[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (po[mid] <= k)
                lo = mid;
            else
                hi = mid;
        }
        s = 1 + lo;
        y = yp;
        nn = np_;
        ns = mp;
        li = k - po[lo];
        n = po[lo + 1] - po[lo];
        start = m0 + po[lo];
        w = wp[k];
    }
    for (int c = 0; c < 3; ++c) {
        const double yc = y[c * ns + k], nc = nn[c * ns + k];
        T[c * ms + i] = yc;
        NS[c * ms + i] = nc;
        bx[3 * start + c * n + li] = yc;
        bn[3 * start + c * n + li] = nc;
    }
    bw[i] = w;
    sid[i] = s;
    self[i] = i;
}

// out = v / d elementwise over 3 n_tot entries.
__global__ __launch_bounds__(PB) void k_pt_scale(int64_t n3, const double* v, const double* d, double* out) {
    const int64_t e = (int64_t)blockIdx.x * PB + threadIdx.x;
    if (e < n3) out[e] = v[e] / d[e];
}

// z = v / diag over the 3 n_tot entries (v given, or v_j = V + j 3 n_tot of the slot
// with j read from the device descriptor when v is null: a replayed iteration advances
// it on the device), and the surface part of z twice: into per-surface SoA blocks qb
// (the moments' input) and, as planes of M_s, into the density of the one
// double-layer sum over all surfaces, with the sign of each surface's term in the
// operator: +q0 on the periphery, -q_p on a particle.
__global__ __launch_bounds__(PB) void k_pt_scale_gather(Surfaces S, int64_t ms, int64_t ntot, const double* v,
                                                        const SlotDesc* D, int slot, const double* diag,
                                                        double* z, double* qb, double* qt) {
    const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
    if (i >= ntot) return;
    if (!v) v = D[slot].V + (int64_t)D[slot].j * 3 * ntot;
    double zc[3];
    for (int c = 0; c < 3; ++c) {
        zc[c] = v[c * ntot + i] / diag[c * ntot + i];
        z[c * ntot + i] = zc[c];
    }
    if (i >= ms) return;
    const int s = S.sid[i];
    const int64_t n = S.ssize[s], li = i - S.sstart[s];
    double* q = qb + 3 * S.sstart[s];
    const double sg = s == 0 ? 1.0 : -1.0;
    for (int c = 0; c < 3; ++c) {
        q[c * n + li] = zc[c];
        qt[c * ms + i] = sg * zc[c];
    }
}

// One block of PR threads per surface, fixed order: area (which = 0) or the moments of
// q (which = 1): periphery red[0] = int n.q0; particle red[8 s + 0..2] = int q,
// red[8 s + 3..5] = int (y - X) x q.
constexpr int PR = 1024;
__global__ __launch_bounds__(PR) void k_pt_reduce(Surfaces S, const double* qb, const double* X, int32_t np,
                                                  int which, double* red) {
    __shared__ double lds[6][PR];
    const int s = blockIdx.x;
    const int t = threadIdx.x;
    const int64_t n = S.ssize[s];
    const double* y = block(S.xyz, S, s);
    const double* nn = block(S.nrm, S, s);
    const double* q = qb + 3 * S.sstart[s];
    const double* w = S.w + S.sstart[s];
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double cx = s > 0 ? X[s - 1] : 0.0, cy = s > 0 ? X[np + s - 1] : 0.0,
                 cz = s > 0 ? X[2 * np + s - 1] : 0.0;
    for (int64_t k = t; k < n; k += PR) {
        if (which == 0) {
            a[0] += w[k];
        } else if (s == 0) {
            a[0] += w[k] * (nn[k] * q[k] + nn[n + k] * q[n + k] + nn[2 * n + k] * q[2 * n + k]);
        } else {
            const double qx = q[k], qy = q[n + k], qz = q[2 * n + k];
            const double rx = y[k] - cx, ry = y[n + k] - cy, rz = y[2 * n + k] - cz;
            a[0] += w[k] * qx;
            a[1] += w[k] * qy;
            a[2] += w[k] * qz;
            a[3] += w[k] * (ry * qz - rz * qy);
            a[4] += w[k] * (rz * qx - rx * qz);
            a[5] += w[k] * (rx * qy - ry * qx);
        }
    }
    for (int c = 0; c < 6; ++c) lds[c][t] = a[c];
    __syncthreads();
    for (int h = PR / 2; h > 0; h >>= 1) {
        if (t < h)
            for (int c = 0; c < 6; ++c) lds[c][t] += lds[c][t + h];
        __syncthreads();
    }
    if (t < 6) red[8 * s + t] = lds[t][0];
}

// w = A z from the double-layer sum Dq = K0[q0] - sum_p K_p[q_p] at every surface point
// (each surface's own term in principal value), the moments red and the areas
// (area[8 s], as k_pt_reduce lays them out).
__global__ __launch_bounds__(PB) void k_pt_assemble(Surfaces S, int64_t ms, int64_t ntot, int32_t np,
                                                    const double* z, const double* Dq, const double* red,
                                                    const double* area, const double* X, double* w) {
    const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
    if (i >= ntot) return;
    double v[3];
    if (i < ms) {
        const int s = S.sid[i];
        for (int c = 0; c < 3; ++c)
            v[c] = -0.5 * z[c * ntot + i] + Dq[c * ms + i];
        const int64_t n = S.ssize[s], li = i - S.sstart[s];
        if (s == 0) {
            const double* nn = block(S.nrm, S, 0);
            for (int c = 0; c < 3; ++c) v[c] += nn[c * n + li] * red[0];
        } else {
            const int p = s - 1;
            const double* y = block(S.xyz, S, s);
            const double rx = y[li] - X[p], ry = y[n + li] - X[np + p], rz = y[2 * n + li] - X[2 * np + p];
            const double ux = z[ms + p], uy = z[ntot + ms + p], uz = z[2 * ntot + ms + p];
            const double ox = z[ms + np + p], oy = z[ntot + ms + np + p], oz = z[2 * ntot + ms + np + p];
            v[0] -= ux + (oy * rz - oz * ry);
            v[1] -= uy + (oz * rx - ox * rz);
            v[2] -= uz + (ox * ry - oy * rx);
        }
    } else {
        const int64_t r = i - ms;
        const int p = (int)(r < np ? r : r - np);
        const int off = r < np ? 0 : 3;
        for (int c = 0; c < 3; ++c)
            v[c] = red[8 * (1 + p) + off + c] / area[8 * (1 + p)] - z[c * ntot + i];
    }
    w[i] = v[0];
    w[ntot + i] = v[1];
    w[2 * ntot + i] = v[2];
}

inline unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + PB - 1) / PB); }

// Device scratch of one solve, freed at the end of the call.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

// Two captured graphs, their executables and the stream they were captured on,
// destroyed with the object.
struct GraphGuard {
    hipStream_t cap = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    ~GraphGuard() {
        for (int p = 0; p < 2; ++p) {
            if (exec[p]) (void)hipGraphExecDestroy(exec[p]);
            if (graph[p]) (void)hipGraphDestroy(graph[p]);
        }
        if (cap) (void)hipStreamDestroy(cap);
    }
};

}  // namespace pt
}  // namespace stokes

using namespace stokes;
using namespace stokes::pt;

extern "C" int stokes_particle_solve(int64_t m0, const double* y0, const double* n0, const double* w0,
                                     int32_t n_part, const int64_t* part_offset, const double* yp,
                                     const double* np_, const double* wp, const double* centers,
                                     const double* force, const double* torque, double mu,
                                     double near_r, int32_t iters, uint32_t flags, double* U_out,
                                     double* Omega_out, double* q_out, double* resid_out,
                                     int32_t* iters_out, void* stream) {
    if (flags & ~(STOKES_PREC_MIXED | STOKES_EAGER))
        return fail(STOKES_E_INVAL, "stokes_particle_solve: unknown flag bits");
    const bool graph = !(flags & STOKES_EAGER);
    if (m0 < 0 || n_part < 1 || !part_offset)
        return fail(STOKES_E_INVAL, "stokes_particle_solve: need m0 >= 0, n_part >= 1 and part_offset");
    if (iters < 1 || iters > STOKES_MAX_ITERS) return fail(STOKES_E_INVAL, "stokes_particle_solve: iters out of range");
    if (!(mu > 0.0)) return fail(STOKES_E_INVAL, "stokes_particle_solve: mu must be > 0");
    if (part_offset[0] != 0) return fail(STOKES_E_INVAL, "stokes_particle_solve: part_offset[0] must be 0");
    for (int p = 0; p < n_part; ++p)
        if (part_offset[p + 1] - part_offset[p] < 4)
            return fail(STOKES_E_INVAL, "stokes_particle_solve: every particle needs >= 4 surface points");
    const int64_t mp = part_offset[n_part];
    const int64_t ms = m0 + mp, ntot = ms + 2 * (int64_t)n_part, n3 = 3 * ntot;
    if (ntot >= ((int64_t)1 << 30)) return fail(STOKES_E_INVAL, "stokes_particle_solve: too many points");
    if ((m0 > 0 && (!y0 || !n0 || !w0)) || !yp || !np_ || !wp || !centers || !force || !torque ||
        !U_out || !Omega_out)
        return fail(STOKES_E_INVAL, "stokes_particle_solve: null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n_surf = 1 + n_part;
    Range range("stokes_particle_solve");
    const uint32_t sumflags = flags & STOKES_PREC_MIXED;

    // host table: surface starts and sizes (Surfaces), then part_offset
    std::vector<int64_t> tab(2 * (size_t)n_surf + n_part + 1);
    tab[0] = 0;
    tab[n_surf] = m0;
    for (int p = 0; p < n_part; ++p) {
        tab[1 + p] = m0 + part_offset[p];
        tab[n_surf + 1 + p] = part_offset[p + 1] - part_offset[p];
    }
    for (int p = 0; p <= n_part; ++p) tab[2 * n_surf + p] = part_offset[p];

    // device scratch
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_T = take(3 * ms * 8), o_N = take(3 * ms * 8), o_bx = take(3 * ms * 8),
                 o_bn = take(3 * ms * 8), o_bw = take(ms * 8), o_sid = take(ms * 4), o_tab = take(tab.size() * 8),
                 o_self = take(ms * 8), o_qt = take(3 * ms * 8), o_qb = take(3 * ms * 8),
                 o_Dq = take(3 * ms * 8), o_red = take(8 * n_surf * 8), o_area = take(8 * n_surf * 8),
                 o_diag = take(n3 * 8), o_rhs = take(n3 * 8), o_slot = take(vector_plan_bytes(ntot, iters));
    DevBuf buf;
    STOKES_HIP(hipMalloc(&buf.p, off));
    char* base = static_cast<char*>(buf.p);
    double* T = reinterpret_cast<double*>(base + o_T);
    double* NS = reinterpret_cast<double*>(base + o_N);
    double* bx = reinterpret_cast<double*>(base + o_bx);
    double* bn = reinterpret_cast<double*>(base + o_bn);
    double* bw = reinterpret_cast<double*>(base + o_bw);
    int32_t* d_sid = reinterpret_cast<int32_t*>(base + o_sid);
    int64_t* d_tab = reinterpret_cast<int64_t*>(base + o_tab);
    int64_t* d_ss = d_tab;
    int64_t* d_sz = d_tab + n_surf;
    const int64_t* d_po = d_tab + 2 * n_surf;
    int64_t* d_self = reinterpret_cast<int64_t*>(base + o_self);
    double* qt = reinterpret_cast<double*>(base + o_qt);
    double* qb = reinterpret_cast<double*>(base + o_qb);
    double* Dq = reinterpret_cast<double*>(base + o_Dq);
    double* red = reinterpret_cast<double*>(base + o_red);
    double* area = reinterpret_cast<double*>(base + o_area);
    double* diag = reinterpret_cast<double*>(base + o_diag);
    double* rhs = reinterpret_cast<double*>(base + o_rhs);
    void* slot = base + o_slot;

    STOKES_HIP(hipMemcpyAsync(d_tab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_pt_geometry, dim3(grid1(ms)), dim3(PB), 0, st, m0, y0, n0, w0, mp, yp, np_, wp, n_part,
                       d_po, T, NS, bx, bn, bw, d_sid, d_self);
    const Surfaces S{bx, bn, bw, d_sid, d_ss, d_sz};

    hipLaunchKernelGGL(k_pt_rhs, dim3(grid1(ntot)), dim3(PB), 0, st, ms, ntot, T, n_part, centers, force,
                       torque, mu, rhs);
    hipLaunchKernelGGL(k_pt_diag, dim3((unsigned)ntot), dim3(64), 0, st, S, ms, ntot, diag);
    hipLaunchKernelGGL(k_pt_reduce, dim3(n_surf), dim3(PR), 0, st, S, (const double*)qb, centers, n_part, 0,
                       area);
    STOKES_HIP(hipGetLastError());

    // The double layers of the operator, K0[q0] - sum_p K_p[q_p] at every surface point,
    // as one sum over all surfaces with the density +q0 on the periphery and -q_p on the
    // particles: each target subtracts its own density (the principal value) only from
    // the sources of its own surface (surface ids d_sid: 0 the periphery, 1 + p the
    // particles) and sums the other surfaces raw.  Tiles, packs and exclusion ranges are
    // made once here; an iteration re-packs only the density.
    DLPlan plan;
    if (int rc = plan.init(ms, T, NS, bw, d_sid, ms, T, d_self, near_r, sumflags, st)) return rc;

    // w = A P^{-1} v on stream s: z = v / diag (v given, or v_j of slot 0 read on the
    // device when v is null: the captured iteration), then the operator
    Batch b;
    auto apply = [&](const double* v, double* z, double* w, hipStream_t s) -> int {
        hipLaunchKernelGGL(k_pt_scale_gather, dim3(grid1(ntot)), dim3(PB), 0, s, S, ms, ntot, v,
                           (const SlotDesc*)b.dev_desc(), 0, (const double*)diag, z, qb, qt);
        if (int rc = plan.eval(qt, Dq, false, s, v == nullptr)) return rc;
        hipLaunchKernelGGL(k_pt_reduce, dim3(n_surf), dim3(PR), 0, s, S, (const double*)qb, centers, n_part,
                           1, red);
        hipLaunchKernelGGL(k_pt_assemble, dim3(grid1(ntot)), dim3(PB), 0, s, S, ms, ntot, n_part,
                           (const double*)z, (const double*)Dq, (const double*)red, (const double*)area,
                           centers, w);
        STOKES_HIP(hipGetLastError());
        return STOKES_OK;
    };

    int rc = b.init(st, false, true, false);
    if (rc) return rc;
    if ((rc = b.attach_vector(0, slot, ntot, iters, rhs))) return rc;
    const std::vector<int> one{0};
    if ((rc = b.start_vector(one))) return rc;
    int done = 0;
    double resid = b.status(0)[2];
    // The iteration -- operator, Gram-Schmidt and the copy of the status row, eleven
    // kernels and a copy -- is captured into a HIP graph and replayed (no memset nodes;
    // v_j and the iteration counter are read on the device, and the last Gram-Schmidt
    // kernel advances the counter), so the host launches one graph per iteration instead
    // of twelve operations whose launch gaps were longer than most of their run times.
    // Two graphs, one per status row, alternate (iteration j copies into row j mod 2).
    // The capture runs on a stream of its own (the caller's may be the null stream, which
    // cannot capture); it only records, and the graphs are replayed on the caller's stream.
    GraphGuard gg;
    if (graph && b.status(0)[3] == 0.0) {
        b.desc(0).j = 0;
        if ((rc = b.ortho_lists(one))) return rc;
        STOKES_HIP(hipStreamCreateWithFlags(&gg.cap, hipStreamNonBlocking));   // (default priority)
        for (int p = 0; p < 2; ++p) {
            STOKES_HIP(hipStreamBeginCapture(gg.cap, hipStreamCaptureModeThreadLocal));
            rc = apply(nullptr, b.desc(0).z, b.desc(0).w, gg.cap);
            if (!rc) rc = b.launch_ortho_fixed(one, gg.cap);
            if (!rc) rc = b.copy_status_async(b.lag_row(p), gg.cap);
            hipGraph_t gr = nullptr;
            const hipError_t e = hipStreamEndCapture(gg.cap, &gr);
            gg.graph[p] = gr;
            if (rc) return rc;
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            STOKES_HIP(hipGraphInstantiate(&gg.exec[p], gg.graph[p], nullptr, nullptr, 0));
        }
    }
    if (b.status(0)[3] == 0.0) {
        // The host does not wait for each iteration: iteration j is enqueued before the
        // status of iteration j - 1 is read (two pinned status rows, one event each).  An
        // exact breakdown is therefore seen one iteration late; the extra iteration then
        // writes only Krylov entries beyond the ones the solution uses (x = 0 input).
        hipError_t e = hipSuccess;
        bool broke = false;
        for (int j = 0; j <= iters && !broke; ++j) {
            if (j < iters) {
                if (graph) {   // the replay computes iteration j (its counter is on the device)
                    const hipError_t ge = hipGraphLaunch(gg.exec[j & 1], st);
                    if (ge != hipSuccess) rc = hip_fail(ge, "hipGraphLaunch");
                } else {
                    SlotDesc& d = b.desc(0);
                    d.j = j;
                    if (!rc) rc = apply(d.V + (int64_t)j * n3, d.z, d.w, st);
                    if (!rc) rc = b.step_ortho_nowait(one);
                    if (!rc) rc = b.copy_status_async(b.lag_row(j));
                }
                if (!rc) {
                    e = hipEventRecord(b.lag_event(j), st);
                    if (e != hipSuccess) rc = hip_fail(e, "hipEventRecord");
                }
            }
            if (j > 0 && !rc) {   // the previous iteration's status
                e = hipEventSynchronize(b.lag_event(j - 1));
                if (e != hipSuccess) rc = hip_fail(e, "hipEventSynchronize");
                if (!rc) {
                    const double* row = b.lag_row(j - 1);
                    done = j;
                    resid = row[2];
                    broke = row[3] != 0.0;   // exact breakdown at iteration j - 1
                }
            }
            if (rc) break;
        }
        if (!rc) {
            e = hipStreamSynchronize(st);   // a late breakdown's extra iteration is done
            if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
        }
        if (rc) return rc;
    }
    b.desc(0).j = done;
    if ((rc = b.finalize_vector(one))) return rc;
    SlotDesc& d = b.desc(0);
    hipLaunchKernelGGL(k_pt_scale, dim3(grid1(n3)), dim3(PB), 0, st, n3, (const double*)d.w,
                       (const double*)diag, d.x);
    STOKES_HIP(hipGetLastError());
    for (int c = 0; c < 3; ++c) {
        STOKES_HIP(hipMemcpyAsync(U_out + c * n_part, d.x + c * ntot + ms, n_part * 8, hipMemcpyDeviceToDevice, st));
        STOKES_HIP(hipMemcpyAsync(Omega_out + c * n_part, d.x + c * ntot + ms + n_part, n_part * 8,
                                  hipMemcpyDeviceToDevice, st));
        if (q_out) STOKES_HIP(hipMemcpyAsync(q_out + c * ms, d.x + c * ntot, ms * 8, hipMemcpyDeviceToDevice, st));
    }
    STOKES_HIP(hipStreamSynchronize(st));
    if (resid_out) *resid_out = resid;
    if (iters_out) *iters_out = done;
    return STOKES_OK;
}
