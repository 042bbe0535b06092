"""Oracle for one implicit (backward Euler) time step of free elastic fibers, following
the section "Time discretization": the Chebyshev fiber representation (section "Fiber
representation"), the fiber force f+ = -E D_s^4 X+ + D_s(T+ X_s), the inextensibility
constraint of eq. inextensibility-mod with the time derivative replaced by its
backward-Euler quotient, the free-end boundary conditions of eq. bc-free, and the
slender-body evolution eq. main-sb-local with the complementary flow of the other
fibers treated implicitly.  Fixed lengths (no polymerisation), no rigid bodies, no
periphery.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Unknowns per fiber with n = p + 1 CGL nodes alpha_k = cos(k pi / p) (node 0 is the plus
end s = L, alpha = 1): X+ (3 n) and T+ (n).  With
  V[f] = M f (+ K_delta f) + u_bar[f]   (u_bar: the other fibers' Stokeslet + doublet sum
                                          with Clenshaw-Curtis weights x L/2)
the position equations are those of eq. discrete-update,

  X+ / dt - V[f+] = X / dt + V[f_ext],   f+ = -E X+_ssss + (T+ X_s)_s,

and the tension equation is the inextensibility constraint in the velocity form the
paper states it in (eq. main-inextensibility), t . (V[f+ + f_ext])_s = 0, written as the
second-order equation for T that the paper takes from Tornberg and Shelley (2004).
Split V = A f + R[f] into the part that acts node by node, A = alpha I + beta t t (M, and
with the nonlocal term its subtracted local part -(8 pi mu)^-1 sum_k w_k psi_ik (I + t t)),
and R (the other fibers' flow and the rest of K_delta, smooth along the fiber).  For
a curve parametrised by arclength (t . X_ss = 0, t . X_sss = -|X_ss|^2,
t . X_ssss = -3 X_ss . X_sss), with c = alpha + beta,

  t . (A f)_s = c_s (t . f) + c (t . f)_s - alpha X_ss . f,
  t . f+      = 3 E X_ss . X+_sss + T_s,
  (t . f+)_s  = 3 E (X_sss . X+_sss + X_ss . X+_ssss) + T_ss,
  X_ss . f+   = -E X_ss . X+_ssss + |X_ss|^2 T,

geometry (t, X_ss, X_sss) explicit and X+, T implicit (section "Time discretization").
The tension equation is then h(X+, T) + t . (R[f+])_s = -t . (V[f_ext])_s with h the
three terms above: fourth order in X and second in T, as the paper counts them.  (The
velocity form differentiated as it stands puts D^5 on X+: such a system has
node-to-node oscillating tension modes.)  The paper leaves open how the boundary
conditions enter the collocation system; here by rectangular collocation (Driscoll and
Hale, IMA J. Numer. Anal. 2016): each position component is collocated at the n - 4
first-kind Chebyshev points (the node values interpolated there) and completed by
X_ss = 0 and X_sss = 0 at both ends; the tension equation is collocated at the n - 2
first-kind points and completed by T = 0 at both ends (eq. bc-free).

A fiber may instead have its minus end (s = 0) attached to a body at rest (U = Ω = 0).
Clamped: eq. BC2-1 and eq. BC2-2 keep that end's position and tangent (X+ = X,
X+_s = X_s there).  Hinged: the position is kept and the end is torque free
(X+ = X, X+_ss = 0, the condition stated beside eq. BC2-2).  Either way eq. BC2-T, the tangential component of the velocity
condition, becomes t . V[f+ + f_ext] = 0 at the end, with t . f+ written as in the
tension equation.

Row layout of the operator (3 N position rows, then N tension rows, fiber by fiber):
position rows of a fiber = its n - 4 collocated rows, then X_ss(s=L), X_sss(s=L),
X_ss(s=0), X_sss(s=0) (clamped: X+(s=0), X+_s(s=0); hinged: X+(s=0), X+_ss(s=0));
tension rows = its n - 2
collocated rows, then T(s=L), T(s=0) (clamped: -t . V[f+](s=0)).
"""
from __future__ import annotations

import math

import numpy as np


def cheb_diff(p):
    """Differentiation on the CGL nodes alpha_k = cos(k pi / p), k = 0..p, in barycentric
    form: D_ij = (w_j / w_i) / (a_i - a_j) for i != j and D_ii = -sum_{j != i} D_ij, with
    w_j = (-1)^j halved at both ends.  Exact for polynomials of degree <= p."""
    k = np.arange(p + 1)
    a = np.cos(k * np.pi / p)
    w = (-1.0) ** k
    w[0] *= 0.5
    w[-1] *= 0.5
    D = np.zeros((p + 1, p + 1))
    for i in range(p + 1):
        for j in range(p + 1):
            if i != j:
                D[i, j] = (w[j] / w[i]) / (a[i] - a[j])
        D[i, i] = -np.sum(D[i, np.arange(p + 1) != i])
    return D


def first_kind_points(m):
    """The m Chebyshev points of the first kind cos((2j + 1) pi / (2 m)), j = 0..m-1."""
    return np.cos((2.0 * np.arange(m) + 1.0) * np.pi / (2.0 * m))


def cheb_resample(p, m):
    """Values at the p + 1 CGL nodes -> values of their interpolant at the m first-kind
    points (barycentric interpolation; a point that coincides with a node copies it)."""
    k = np.arange(p + 1)
    a = np.cos(k * np.pi / p)
    w = (-1.0) ** k
    w[0] *= 0.5
    w[-1] *= 0.5
    y = first_kind_points(m)
    P = np.zeros((m, p + 1))
    for j in range(m):
        d = y[j] - a
        hit = np.flatnonzero(d == 0.0)
        if hit.size:
            P[j, hit[0]] = 1.0
            continue
        c = w / d
        P[j] = c / np.sum(c)
    return P


class FiberStep:
    """The linear system of one backward-Euler step for free fibers: current geometry X
    (3, N) fiber-contiguous with `npf` nodes per fiber, lengths L (n_fib,), slenderness
    eps, bending modulus E, step dt, viscosity mu, optional nonlocal term (delta), and
    the source doublet in the other fibers' flow (doublet)."""

    def __init__(self, X, L, npf, eps, E, dt, mu=1.0, delta=None, doublet=True, nthreads=1,
                 clamp=None):
        self.X = np.asarray(X, dtype=np.float64)
        self.L = np.asarray(L, dtype=np.float64)
        self.npf, self.eps, self.E, self.dt, self.mu = npf, eps, E, dt, mu
        self.delta, self.doublet, self.nthreads = delta, doublet, nthreads
        self.N = self.X.shape[1]
        self.nf = self.N // npf
        assert self.nf * npf == self.N and self.L.size == self.nf and npf >= 6
        self.fib = np.repeat(np.arange(self.nf), npf)
        # minus-end condition per fiber: 0 free, 1 clamped, 2 hinged (to a body at rest)
        self.clamp = np.zeros(self.nf, int) if clamp is None else np.asarray(clamp, int).ravel()
        assert self.clamp.size == self.nf and np.all((self.clamp >= 0) & (self.clamp <= 2))
        p = npf - 1
        self.Da = cheb_diff(p)
        self.P4 = cheb_resample(p, npf - 4)
        self.P2 = cheb_resample(p, npf - 2)
        self.D2 = self.Da @ self.Da
        self.D3 = self.D2 @ self.Da
        self.D4 = self.D3 @ self.Da
        self.Xa = self.per_fiber(self.Da, self.X, 0)
        self.Xs = self.Xa * (2.0 / self.L[self.fib])[None, :]
        self.tangent = self.Xs / np.linalg.norm(self.Xs, axis=0)
        self.Xss = self.per_fiber(self.D2, self.X, 2)
        self.Xsss = self.per_fiber(self.D3, self.X, 3)
        # the node-by-node part A = alpha I + beta t t of V, and c = alpha + beta
        pref = 1.0 / (8.0 * math.pi * mu)
        kap = -math.log(eps * eps * math.e)
        self.alpha = np.full(self.N, pref * (kap + 2.0))
        self.c = np.full(self.N, pref * 2.0 * kap)
        if delta is not None:
            import oracle
            w = oracle.fiber_quadrature_weights(self.fib, self.L, npf)
            sa = oracle.fiber_arclength(self.fib, self.L, npf)
            self.dsum = np.zeros(self.N)
            for i in range(self.N):
                ks = np.arange((i // npf) * npf, (i // npf + 1) * npf)
                ks = ks[ks != i]
                self.dsum[i] = np.sum(w[ks] / np.sqrt((sa[i] - sa[ks]) ** 2 + delta * delta))
            self.alpha -= pref * self.dsum
            self.c -= 2.0 * pref * self.dsum
        self.c_s = self.per_fiber(self.Da, self.c[None, :], 1)[0]

    def per_fiber(self, A, V, scale_pow):
        """Apply the matrix A (rows x n) on each fiber to V (c, N) times (2/L)^scale_pow;
        returns (c, n_fib * rows)."""
        r = A.shape[0]
        out = np.zeros(V.shape[:-1] + (self.nf * r,))
        for m in range(self.nf):
            sl = slice(m * self.npf, (m + 1) * self.npf)
            out[..., m * r:(m + 1) * r] = V[..., sl] @ A.T * (2.0 / self.L[m]) ** scale_pow
        return out

    def force(self, Xp, T):
        """f+ = -E D_s^4 X+ + D_s (T+ X_s), with X_s of the current geometry."""
        return (-self.E * self.per_fiber(self.D4, Xp, 4)
                + self.per_fiber(self.Da, T[None, :] * self.Xs, 1))

    def smooth_velocity(self, f, others=True):
        """R[f] = V[f] - A f: the other fibers' flow and K_delta without its subtracted
        local part."""
        import oracle
        v = np.zeros_like(f)
        if self.delta is not None:
            t = self.tangent
            proj = f + t * np.sum(t * f, axis=0)
            v = (oracle.nonlocal_sbt(f, self.X, t, self.fib, self.L, self.npf, self.delta, self.mu)
                 + proj * (self.dsum / (8.0 * math.pi * self.mu))[None, :])
        if others:
            w = oracle.fiber_quadrature_weights(self.fib, self.L, self.npf)
            v = v + oracle.sl(self.X, f, src_weight=w, src_fiber=self.fib, fiber_len=self.L,
                              mu=self.mu, eps=self.eps, excl=oracle.EXCL_SAME_FIBER,
                              doublet=self.doublet, nthreads=self.nthreads)
        return v

    def tension_local(self, Xp, T):
        """h(X+, T): t . (A f+)_s with the arclength identities (module docstring)."""
        E = self.E
        x3 = self.per_fiber(self.D3, Xp, 3)
        x4 = self.per_fiber(self.D4, Xp, 4)
        Ts = self.per_fiber(self.Da, T[None, :], 1)[0]
        Tss = self.per_fiber(self.D2, T[None, :], 2)[0]
        ss3 = np.sum(self.Xss * x3, axis=0)
        ss4 = np.sum(self.Xss * x4, axis=0)
        sss3 = np.sum(self.Xsss * x3, axis=0)
        k2 = np.sum(self.Xss * self.Xss, axis=0)
        tf = 3.0 * E * ss3 + Ts
        tf_s = 3.0 * E * (sss3 + ss4) + Tss
        ssf = -E * ss4 + k2 * T
        return self.c_s * tf + self.c * tf_s - self.alpha * ssf

    def t_dot_ds(self, v):
        """t . (v)_s at the nodes (D_s on node values)."""
        return np.sum(self.tangent * self.per_fiber(self.Da, v, 1), axis=0)

    def local_velocity(self, f):
        """A f: M f, and with the nonlocal term its subtracted local part
        -(8 pi mu)^-1 sum_k w_k psi_ik (I + t t) f (eq. main-sb-local, eq. sb-stokes-reg)."""
        import oracle
        v = oracle.local_sbt(f, self.tangent, self.eps, self.mu)
        if self.delta is not None:
            t = self.tangent
            v = v - (f + t * np.sum(t * f, axis=0)) * (self.dsum / (8.0 * math.pi * self.mu))[None, :]
        return v

    def velocity(self, f, others=True):
        """V[f] = M f (+ K_delta f) (+ the flow of the other fibers at the nodes)."""
        return self.local_velocity(f) + self.smooth_velocity(f, others)

    def _assemble(self, pos_nodes, ten_nodes, bc_pos, bc_ten):
        """Collocate node values and append the boundary rows (row layout: module doc)."""
        n = self.npf
        pos = np.zeros((3, self.N))
        ten = np.zeros(self.N)
        for m in range(self.nf):
            o = m * n
            sl = slice(o, o + n)
            pos[:, o:o + n - 4] = pos_nodes[:, sl] @ self.P4.T
            pos[:, o + n - 4:o + n] = bc_pos[:, 4 * m:4 * m + 4]
            ten[o:o + n - 2] = self.P2 @ ten_nodes[sl]
            ten[o + n - 2:o + n] = bc_ten[2 * m:2 * m + 2]
        return np.concatenate([pos.ravel(), ten])

    def apply(self, Y, others=True):
        """The step's linear operator on Y = [X+ (3 N, component-major) | T+ (N)]."""
        Y = np.asarray(Y, dtype=np.float64).ravel()
        Xp = Y[: 3 * self.N].reshape(3, self.N)
        T = Y[3 * self.N:]
        f = self.force(Xp, T)
        pos = Xp / self.dt - self.local_velocity(f) - (vr := self.smooth_velocity(f, others))
        ten = -(self.tension_local(Xp, T) + self.t_dot_ds(vr))
        p = self.npf - 1
        s1 = self.per_fiber(self.Da, Xp, 1)
        s2 = self.per_fiber(self.D2, Xp, 2)
        s3 = self.per_fiber(self.D3, Xp, 3)
        # clamped minus end: t . V[f+] there, with t . f+ = 3 E X_ss . X+_sss + T_s
        tf = 3.0 * self.E * np.sum(self.Xss * s3, axis=0) + self.per_fiber(self.Da, T[None, :], 1)[0]
        tv = self.c * tf + np.sum(self.tangent * vr, axis=0)
        bc_pos = np.zeros((3, 4 * self.nf))
        bc_ten = np.zeros(2 * self.nf)
        for m in range(self.nf):
            o = m * self.npf
            if self.clamp[m]:
                second = s1[:, o + p] if self.clamp[m] == 1 else s2[:, o + p]
                bc_pos[:, 4 * m:4 * m + 4] = np.stack([s2[:, o], s3[:, o], Xp[:, o + p], second], axis=1)
                bc_ten[2 * m:2 * m + 2] = [T[o], -tv[o + p]]
            else:
                bc_pos[:, 4 * m:4 * m + 4] = np.stack([s2[:, o], s3[:, o], s2[:, o + p], s3[:, o + p]],
                                                      axis=1)
                bc_ten[2 * m:2 * m + 2] = [T[o], T[o + p]]
        return self._assemble(pos, ten, bc_pos, bc_ten)

    def rhs(self, fext):
        v = self.velocity(np.asarray(fext, dtype=np.float64))
        pos = self.X / self.dt + v
        ten = self.t_dot_ds(v)
        bc_pos = np.zeros((3, 4 * self.nf))
        bc_ten = np.zeros(2 * self.nf)
        p = self.npf - 1
        tv = np.sum(self.tangent * v, axis=0)
        for m in range(self.nf):
            if self.clamp[m]:     # the end keeps its position (and tangent), no tangential velocity
                o = m * self.npf
                bc_pos[:, 4 * m + 2] = self.X[:, o + p]
                if self.clamp[m] == 1:
                    bc_pos[:, 4 * m + 3] = self.Xs[:, o + p]
                bc_ten[2 * m + 1] = tv[o + p]
        return self._assemble(pos, ten, bc_pos, bc_ten)

    def self_blocks(self):
        """Per fiber, the operator without the other fibers' flow as a 4n x 4n matrix
        (unknowns and rows ordered x, y, z, T, each over the fiber's n slots)."""
        n = self.npf
        blocks = []
        for m in range(self.nf):
            sub = type(self)(self.X[:, m * n:(m + 1) * n], self.L[m:m + 1], n, self.eps, self.E,
                             self.dt, self.mu, self.delta, self.doublet, clamp=self.clamp[m:m + 1])
            blocks.append(np.stack([sub.apply(e, others=False) for e in np.eye(4 * n)], axis=1))
        return blocks

    def block_index(self, m):
        n, N = self.npf, self.N
        return np.concatenate([c * N + m * n + np.arange(n) for c in range(4)])

    def precond(self, blocks):
        """Block-Jacobi: solve each fiber's self block (section "Linear solver and
        preconditioner")."""
        def Pinv(v):
            v = np.asarray(v).ravel()
            out = np.empty_like(v)
            for m, B in enumerate(blocks):
                idx = self.block_index(m)
                out[idx] = np.linalg.solve(B, v[idx])
            return out
        return Pinv


def fiber_step(X, L, npf, eps, E, dt, fext, iters, mu=1.0, delta=None, doublet=True, clamp=None):
    """One step by right-preconditioned GMRES with the fiber block-Jacobi preconditioner
    (section "Linear solver and preconditioner").  The unknown is the increment
    (X+ - X, T+): the same linear system shifted by the current geometry,
    A [dX, T] = b - A [X, 0], so that rounding scales with one step's motion and not
    with the coordinates (the operator amplifies node rounding by up to p^10 through the
    tension rows).  Returns (X+ (3, N), T+ (N,), residual history, iterations)."""
    from oracle import gmres
    S = FiberStep(X, L, npf, eps, E, dt, mu, delta, doublet, clamp=clamp)
    N = S.N
    b = S.rhs(fext) - S.apply(np.concatenate([S.X.ravel(), np.zeros(N)]))
    y, hist, m = gmres(S.apply, b, iters, S.precond(S.self_blocks()))
    return S.X + y[: 3 * N].reshape(3, N), y[3 * N:], hist, m
