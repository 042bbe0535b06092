"""Oracle for confined rigid particles: the second-kind boundary integral mobility
problem of sections "The contribution from the periphery" and "The contribution from
rigid immersed particles" (eq. main-cortex-density, eq. main-nsb-second-kind,
eq. main-nsb-rgbt, eq. main-nsb-rgbr), discretised by Nystrom on the given surface
quadrature, with singularity subtraction on the surfaces and the diagonal Jacobi
preconditioner of eq. prec.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions.  K[q](x) = (3/(4 pi)) sum_s w_s (d.q_s)(d.n_s) d / |d|^5, d = x - y_s, n
OUTWARD, is the double-layer sum of ``oracle.dl`` (its on-surface value, with
``subtract``, is the principal value).  The paper's double layer with the normal
pointing into the fluid is K itself on the periphery (fluid inside) and -K on a
particle (fluid outside).  With that, for no-slip on a fixed periphery Gamma_0 and
rigid particles P_p moved by external forces F_p and torques L_p:

  x on Gamma_0:  -q0/2 + K0_PV[q0] + n(x) int n.q0 dS - sum_p K_p[q_p] = -sum_p u_p^ext(x)
  x on P_p:      -q_p/2 - K_p,PV[q_p] - sum_{p' != p} K_p'[q_p'] + K0[q0]
                 - U_p - Omega_p x (x - X_p)                      = -sum_p' u_p'^ext(x)
  (1/|P_p|) int q_p dS - U_p = 0,   (1/|P_p|) int (y - X_p) x q_p dS - Omega_p = 0

with u_p^ext(x) = G(x - X_p) F_p + R(x - X_p) L_p (eq. oseen, eq. rotlet).

Unknown vector: three planes of Ntot = M0 + sum M_p + 2 n_p entries,
[q0 | q_1 ... q_np | U_1 ... U_np | Omega_1 ... Omega_np] per component.
"""
from __future__ import annotations

import math

import numpy as np


def stokeslet(r, F, mu):
    """G(r) F = (F/|r| + r (r.F)/|r|^3) / (8 pi mu), r (3, n), F (3,)."""
    rn = np.sqrt(np.sum(r * r, axis=0))
    rF = np.sum(r * F[:, None], axis=0)
    return (F[:, None] / rn + r * (rF / rn ** 3)) / (8.0 * math.pi * mu)


def rotlet(r, L, mu):
    """R(r) L = (L x r) / (8 pi mu |r|^3)."""
    rn = np.sqrt(np.sum(r * r, axis=0))
    return np.cross(L[:, None], r, axis=0) / rn ** 3 / (8.0 * math.pi * mu)


def dl_diagonal(y, n, w):
    """sum_{s != i} w_s K_cc(y_i - y_s), the coefficient of q_i,c in the singular part of
    the subtracted double-layer sum at y_i, for every point i and component c."""
    y = np.asarray(y, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    m = y.shape[1]
    out = np.zeros((3, m))
    for i in range(m):
        d = y[:, i:i + 1] - y
        r2 = np.sum(d * d, axis=0)
        r2[i] = 1.0
        dn = np.sum(d * n, axis=0)
        k = 3.0 / (4.0 * math.pi) * w * dn / r2 ** 2.5
        k[i] = 0.0
        out[:, i] = np.sum(k[None, :] * d * d, axis=1)
    return out


class ParticleSystem:
    """Periphery (may be empty) and rigid particles, all as surface quadratures:
    points (3, M), outward unit normals (3, M), weights (M,); particle centres X_p."""

    def __init__(self, periphery, particles, mu=1.0):
        if periphery is None:
            periphery = (np.zeros((3, 0)), np.zeros((3, 0)), np.zeros(0))
        self.y0, self.n0, self.w0 = (np.asarray(a, dtype=np.float64) for a in periphery)
        self.parts = [tuple(np.asarray(a, dtype=np.float64) for a in p) for p in particles]
        self.mu = mu
        self.M0 = self.y0.shape[1]
        self.Mp = [p[0].shape[1] for p in self.parts]
        self.np = len(self.parts)
        self.off = np.concatenate([[self.M0], self.M0 + np.cumsum(self.Mp)]).astype(int)
        self.Ms = int(self.off[-1])                        # surface points
        self.Ntot = self.Ms + 2 * self.np
        self.T = np.concatenate([self.y0] + [p[0] for p in self.parts], axis=1)

    def u_index(self, p):
        return self.Ms + p

    def o_index(self, p):
        return self.Ms + self.np + p

    def apply(self, x):
        from oracle import dl
        x = np.asarray(x, dtype=np.float64).reshape(3, self.Ntot)
        q = x[:, : self.Ms]
        out = -0.5 * q.copy()
        if self.M0:
            self0 = np.concatenate([np.arange(self.M0), -np.ones(self.Ms - self.M0, dtype=np.int64)])
            out += dl(self.y0, self.n0, self.w0, q[:, : self.M0], trg_xyz=self.T, trg_self=self0,
                      subtract=True)
            s0 = np.sum(self.w0 * np.sum(self.n0 * q[:, : self.M0], axis=0))
            out[:, : self.M0] += self.n0 * s0
        for p, (y, n, w, X) in enumerate(self.parts):
            a, b = self.off[p], self.off[p + 1]
            selfp = -np.ones(self.Ms, dtype=np.int64)
            selfp[a:b] = np.arange(b - a)
            out -= dl(y, n, w, q[:, a:b], trg_xyz=self.T, trg_self=selfp, subtract=True)
            U = x[:, self.u_index(p)]
            Om = x[:, self.o_index(p)]
            out[:, a:b] -= U[:, None] + np.cross(Om[:, None], y - X[:, None], axis=0)
        res = np.zeros((3, self.Ntot))
        res[:, : self.Ms] = out
        for p, (y, n, w, X) in enumerate(self.parts):
            a, b = self.off[p], self.off[p + 1]
            area = np.sum(w)
            qp = q[:, a:b]
            res[:, self.u_index(p)] = np.sum(w * qp, axis=1) / area - x[:, self.u_index(p)]
            res[:, self.o_index(p)] = (np.sum(w * np.cross(y - X[:, None], qp, axis=0), axis=1)
                                       / area - x[:, self.o_index(p)])
        return res

    def rhs(self, F, L):
        F = np.asarray(F, dtype=np.float64).reshape(3, self.np)
        L = np.asarray(L, dtype=np.float64).reshape(3, self.np)
        b = np.zeros((3, self.Ntot))
        for p, (_, _, _, X) in enumerate(self.parts):
            r = self.T - X[:, None]
            b[:, : self.Ms] -= stokeslet(r, F[:, p], self.mu) + rotlet(r, L[:, p], self.mu)
        return b

    def diagonal(self):
        """Diagonal of the self-interaction blocks (eq. prec): -1 - sum w K_cc + w n_c^2 on
        the periphery, sum w K_cc over the own particle on a particle, -1 for U and Omega."""
        d = -np.ones((3, self.Ntot))
        if self.M0:
            d[:, : self.M0] = (-1.0 - dl_diagonal(self.y0, self.n0, self.w0)
                               + self.w0 * self.n0 * self.n0)
        for p, (y, n, w, X) in enumerate(self.parts):
            a, b = self.off[p], self.off[p + 1]
            d[:, a:b] = dl_diagonal(y, n, w)
        return d


def particle_solve(system, F, L, iters):
    """GMRES (right diagonal-Jacobi preconditioner) on the system above.
    Returns (U (3, n_p), Omega (3, n_p), x (3, Ntot), residual history, iterations)."""
    from oracle import gmres
    diag = system.diagonal()

    def A(v):
        return system.apply(v.reshape(3, system.Ntot)).ravel()

    def Pinv(v):
        return (v.reshape(3, system.Ntot) / diag).ravel()

    x, hist, m = gmres(A, system.rhs(F, L).ravel(), iters, Pinv)
    x = x.reshape(3, system.Ntot)
    U = x[:, system.Ms: system.Ms + system.np]
    Om = x[:, system.Ms + system.np:]
    return U, Om, x, hist, m
