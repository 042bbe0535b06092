"""Pins of the oracle's implicit fiber time step (section "Time discretization"): the
Chebyshev operators against numpy's Chebyshev series, and the step against what the
mechanics fixes.

* A straight fiber under a uniform force translates rigidly with M f (eq. main-sb-local)
  and carries no tension, with or without the nonlocal term.
* A straight fiber under a tangential force g(s) t translates with the mean force, and
  its tension solves T_s = <g> - g with T = 0 at both free ends (eq. bc-free).
* A nearly straight fiber bent into a free-free Euler-Bernoulli beam mode (cos(bL)
  cosh(bL) = 1) relaxes in one backward-Euler step by the factor 1/(1 + dt M_nn E b^4).
* At small dt the tension of a planar curve solves the arclength-reduced tension
  equation (a two-point problem solved by scipy).
* A minus end clamped to a body at rest (eq. BC2-1, BC2-2, BC2-T) keeps its position
  and tangent; a clamped straight fiber under a tangential load does not move and its
  tension is the load beyond s; clamped-free beam modes (cos(bL) cosh(bL) = -1) relax
  by 1/(1 + dt M_nn E b^4).
* The step is consistent (one step against two half steps: local error of order above
  one), changes the length by a small fraction of the motion, and is covariant under rotations; fibers far apart decouple; on several
  fibers the block-preconditioned GMRES reaches the dense solution.
"""
import math

import numpy as np
import pytest

cheb = np.polynomial.chebyshev


def cgl(p):
    return np.cos(np.arange(p + 1) * np.pi / p)


def m_coeffs(eps, mu):
    kap = -math.log(eps * eps * math.e)
    return 2.0 * kap / (8 * math.pi * mu), (kap + 2.0) / (8 * math.pi * mu)   # M_tt, M_nn


def straight(p, L, t, c0):
    t = np.asarray(t, float) / np.linalg.norm(t)
    return np.asarray(c0, float)[:, None] + (L / 2) * cgl(p)[None, :] * t[:, None], t


def normal_to(t):
    n = np.cross(t, [0.3, 1.0, -0.2])
    return n / np.linalg.norm(n)


@pytest.mark.parametrize("p", [7, 16, 31])
def test_cheb_diff_exact_on_polynomials(oracle_mod, p):
    rng = np.random.default_rng(p)
    c = rng.standard_normal(p + 1)
    a = cgl(p)
    D = oracle_mod.cheb_diff(p)
    assert np.abs(D @ cheb.chebval(a, c) - cheb.chebval(a, cheb.chebder(c))).max() <= 1e-11 * p ** 2
    assert np.abs(D @ np.ones(p + 1)).max() <= 1e-12 * p ** 2


@pytest.mark.parametrize("p,m", [(15, 11), (15, 13), (16, 12), (16, 15), (31, 29)])
def test_resample_exact_on_polynomials(oracle_mod, p, m):
    from oracle.timestep import cheb_resample, first_kind_points
    rng = np.random.default_rng(p * m)
    c = rng.standard_normal(p + 1)
    y = first_kind_points(m)
    assert np.allclose(np.cos((2 * np.arange(m) + 1) * np.pi / (2 * m)), y)
    P = cheb_resample(p, m)
    assert np.abs(P @ cheb.chebval(cgl(p), c) - cheb.chebval(y, c)).max() <= 1e-12 * p
    assert np.abs(P.sum(axis=1) - 1).max() <= 1e-13


@pytest.mark.parametrize("delta", [None, 0.05])
def test_straight_fiber_uniform_force_translates(oracle_mod, delta):
    p, L, eps, mu, E, dt = 23, 1.3, 0.01, 0.7, 2.0, 1e-3
    X, t = straight(p, L, [0.3, -0.4, 0.866], [0.2, 0.1, -0.3])
    f = np.array([0.4, -1.1, 0.25])
    fE = np.repeat(f[:, None], p + 1, axis=1)
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, fE, 6, mu, delta=delta)
    Mtt, Mnn = m_coeffs(eps, mu)
    U = Mnn * f + (Mtt - Mnn) * t * np.dot(t, f)
    # rounding: the tension rows carry up to the fifth derivative of the nodes (~p^10)
    assert np.abs(Xp - X - dt * U[:, None]).max() <= 1e-6 * dt * np.abs(U).max()
    assert np.abs(T).max() <= 1e-4 * np.abs(f).max() * L


def test_straight_fiber_tangential_force_tension(oracle_mod):
    p, L, eps, mu, E, dt = 20, 1.7, 0.02, 1.1, 0.5, 2e-3
    X, t = straight(p, L, [1.0, 2.0, -0.5], [0.0, 0.3, 0.1])
    s = 0.5 * L * (1 + cgl(p))
    g = s ** 2 - 0.3 * s + 0.2                       # tangential force density
    G = s ** 3 / 3 - 0.15 * s ** 2 + 0.2 * s         # its primitive from s = 0
    C = (L ** 3 / 3 - 0.15 * L ** 2 + 0.2 * L) / L   # mean force per length
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, g[None, :] * t[:, None], 8, mu)
    Mtt, _ = m_coeffs(eps, mu)
    assert np.abs(T - (C * s - G)).max() <= 1e-8 * np.abs(C * s - G).max()
    assert np.abs(Xp - X - dt * Mtt * C * t[:, None]).max() <= 1e-8 * dt * Mtt * C


def beam_mode(bL, x, L):
    b = bL / L
    sig = (math.cosh(bL) - math.cos(bL)) / (math.sinh(bL) - math.sin(bL))
    return np.cosh(b * x) + np.cos(b * x) - sig * (np.sinh(b * x) + np.sin(b * x))


@pytest.mark.parametrize("bL", [4.730040744862704, 7.853204624095838])
def test_free_free_beam_mode_decay(oracle_mod, bL):
    assert abs(math.cos(bL) * math.cosh(bL) - 1) < 1e-9
    p, L, eps, mu, E, dt, A = 31, 1.2, 0.01, 0.9, 1.5, 2e-3, 1e-6
    X0, t = straight(p, L, [0.2, 0.9, 0.4], [0.0, 0.0, 0.0])
    nv = normal_to(t)
    s = 0.5 * L * (1 + cgl(p))
    X = X0 + A * beam_mode(bL, s, L)[None, :] * nv[:, None]
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, np.zeros((3, p + 1)), 8, mu)
    _, Mnn = m_coeffs(eps, mu)
    factor = 1.0 / (1.0 + dt * Mnn * E * (bL / L) ** 4)
    hp = nv @ Xp
    assert 0.05 < factor < 0.95
    assert np.abs(hp - factor * A * beam_mode(bL, s, L)).max() <= 1e-4 * A


def bent(p, L, amp=0.15):
    """A smooth planar shape parametrised by arclength with X_ss = X_sss = 0 at both ends
    (tangent angle theta(s) with theta' and theta'' zero at the ends)."""
    from scipy.integrate import quad
    u = lambda s: s / L
    theta = lambda s: amp * (u(s) ** 3 * (10 - 15 * u(s) + 6 * u(s) ** 2))
    s = 0.5 * L * (1 + cgl(p))
    xs = np.array([quad(lambda q: math.cos(theta(q)), 0, si, epsabs=1e-13, epsrel=1e-13)[0] for si in s])
    ys = np.array([quad(lambda q: math.sin(theta(q)), 0, si, epsabs=1e-13, epsrel=1e-13)[0] for si in s])
    return np.stack([xs, ys, 0.1 * np.ones_like(xs)])


def length(oracle_mod, X, p):
    D = oracle_mod.cheb_diff(p)
    return np.sum(oracle_mod.clenshaw_curtis(p) * np.linalg.norm(X @ D.T, axis=0))


def test_consistent_in_dt_and_length_kept(oracle_mod):
    p, L, eps, mu, E = 24, 1.0, 0.01, 1.0, 1.0
    X = bent(p, L)
    fE = np.repeat(np.array([[0.0], [0.0], [1.0]]), p + 1, axis=1) + 0.5 * X

    def step(X, dt):
        return oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, fE, 10, mu)[0]
    errs = []
    for dt in (2.5e-4, 1.25e-4, 6.25e-5):
        one = step(X, dt)
        two = step(step(X, dt / 2), dt / 2)
        errs.append(np.abs(one - two).max())
        # the length changes by a small fraction of the motion
        assert abs(length(oracle_mod, one, p) - L) <= 1e-2 * np.abs(one - X).max()
    # local error O(dt^2) for smooth data; the end conditions are not compatible with
    # this force, which reduces the observed order to about 1.5 (ratio ~2.8)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 2.4 < r1 < 4.8 and 2.4 < r2 < 4.8, errs


@pytest.mark.parametrize("amp", [0.6, -1.1])
def test_tension_of_a_planar_curve_at_small_dt(oracle_mod, amp):
    """dt -> 0 with f_ext = 0 on one fiber: X+ -> X and the tension solves the
    arclength-reduced tension equation of the current shape, a two-point problem
    c T'' - alpha k^2 T = -3 c E (k'^2 + k k'') - alpha E (k k'' - k^4), T(0) = T(L) = 0,
    for a planar curve of curvature k(s) (|X_sss|^2 = k'^2 + k^4, X_ss . X_ssss =
    k k'' - k^4), c = 2 kappa / (8 pi mu), alpha = (kappa + 2) / (8 pi mu); solved here by
    scipy's collocation BVP solver, independently of the Chebyshev discretisation."""
    from scipy.integrate import solve_bvp
    p, L, eps, mu, E = 31, 1.0, 0.01, 0.8, 1.3
    X = bent(p, L, amp=amp)
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, 1e-9, np.zeros((3, p + 1)), 8,
                                        mu)
    kap = -math.log(eps * eps * math.e)
    c, al = 2 * kap / (8 * math.pi * mu), (kap + 2) / (8 * math.pi * mu)
    k = lambda s: amp * 30 * (s / L) ** 2 * (1 - s / L) ** 2 / L
    k1 = lambda s: amp * 60 * (s / L) * (1 - s / L) * (1 - 2 * s / L) / L ** 2
    k2 = lambda s: amp * 60 * (1 - 6 * s / L + 6 * (s / L) ** 2) / L ** 3

    def rhs(s, y):
        src = -3 * c * E * (k1(s) ** 2 + k(s) * k2(s)) - al * E * (k(s) * k2(s) - k(s) ** 4)
        return np.vstack([y[1], (al * k(s) ** 2 * y[0] + src) / c])
    grid = np.linspace(0, L, 401)
    sol = solve_bvp(rhs, lambda a, b: np.array([a[0], b[0]]), grid, np.zeros((2, grid.size)),
                    tol=1e-8, max_nodes=1000000)
    assert sol.success
    s = 0.5 * L * (1 + cgl(p))
    ref = sol.sol(s)[0]
    assert np.abs(ref).max() > 0.05
    assert np.abs(T - ref).max() <= 1e-5 * np.abs(ref).max()
    assert np.abs(Xp - X).max() <= 1e-6
def test_clamped_straight_fiber_holds_a_tangential_load(oracle_mod):
    # clamped at s = 0, pulled along itself: it cannot move, and the tension carries the
    # load of the part beyond s, T(s) = int_s^L g (eq. BC2-1, BC2-2, BC2-T with U = Omega = 0)
    p, L, eps, mu, E, dt = 20, 1.4, 0.02, 0.8, 1.3, 2e-3
    X, t = straight(p, L, [0.5, -1.0, 0.3], [0.1, 0.0, 0.2])
    s = 0.5 * L * (1 + cgl(p))
    g = s ** 2 - 0.3 * s + 0.2
    G = lambda x: x ** 3 / 3 - 0.15 * x ** 2 + 0.2 * x
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, g[None, :] * t[:, None], 8, mu,
                                        clamp=[True])
    ref = G(L) - G(s)
    assert np.abs(T - ref).max() <= 1e-8 * np.abs(ref).max()
    assert np.abs(Xp - X).max() <= 1e-10


def test_clamped_end_keeps_position_and_tangent(oracle_mod):
    p, L, eps, mu, E, dt = 24, 1.0, 0.01, 1.0, 0.7, 5e-3
    X = bent(p, L)
    fE = np.random.default_rng(2).standard_normal((3, p + 1))
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, fE, 12, mu, clamp=[True])
    D = oracle_mod.cheb_diff(p)
    assert np.abs(Xp - X).max() > 1e-4                            # the fiber moves
    assert np.abs(Xp[:, p] - X[:, p]).max() <= 1e-12              # the clamped node does not
    assert np.abs((Xp - X) @ D[p]).max() <= 1e-10                 # nor its tangent
    Xf, _, _, _ = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, fE, 12, mu)
    assert np.abs(Xf[:, p] - X[:, p]).max() > 1e-4                # free, the same end moves


def clamped_mode(bL, x, L):
    b = bL / L
    sig = (math.cosh(bL) + math.cos(bL)) / (math.sinh(bL) + math.sin(bL))
    return np.cosh(b * x) - np.cos(b * x) - sig * (np.sinh(b * x) - np.sin(b * x))


@pytest.mark.parametrize("bL", [1.8751040687119611, 4.694091132974175])
def test_clamped_free_beam_mode_decay(oracle_mod, bL):
    assert abs(math.cos(bL) * math.cosh(bL) + 1) < 1e-9
    # (amplitude 1e-5: rounding of this system, ~1e-10 absolute at 32 nodes, stays well
    # below the bound, and the neglected nonlinear terms are O(A) relative)
    p, L, eps, mu, E, dt, A = 31, 1.1, 0.01, 0.9, 1.5, 2e-2, 1e-5
    X0, t = straight(p, L, [0.2, 0.9, 0.4], [0.0, 0.0, 0.0])
    nv = normal_to(t)
    s = 0.5 * L * (1 + cgl(p))                                    # s = 0 is the clamped end
    X = X0 + A * clamped_mode(bL, s, L)[None, :] * nv[:, None]
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, np.zeros((3, p + 1)), 8, mu,
                                        clamp=[True])
    _, Mnn = m_coeffs(eps, mu)
    factor = 1.0 / (1.0 + dt * Mnn * E * (bL / L) ** 4)
    assert 0.05 < factor < 0.95
    assert np.abs(nv @ Xp - factor * A * clamped_mode(bL, s, L)).max() <= 1e-3 * A


def hinged_mode(bL, x, L):
    b = bL / L
    return math.sin(bL) * np.sinh(b * x) + math.sinh(bL) * np.sin(b * x)


def test_hinged_free_beam_mode_decay_and_end(oracle_mod):
    # hinged at s = 0 to a body at rest: position kept, torque free (X_ss = 0); the
    # hinged-free modes (tan(bL) = tanh(bL)) relax by 1/(1 + dt M_nn E b^4)
    bL = 3.926602312047919
    assert abs(math.tan(bL) - math.tanh(bL)) < 1e-9
    p, L, eps, mu, E, dt, A = 31, 1.1, 0.01, 0.9, 1.5, 2e-3, 1e-5
    X0, t = straight(p, L, [0.2, 0.9, 0.4], [0.0, 0.0, 0.0])
    nv = normal_to(t)
    s = 0.5 * L * (1 + cgl(p))
    X = X0 + A * hinged_mode(bL, s, L)[None, :] * nv[:, None]
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L]), p + 1, eps, E, dt, np.zeros((3, p + 1)), 8, mu,
                                        clamp=[2])
    _, Mnn = m_coeffs(eps, mu)
    factor = 1.0 / (1.0 + dt * Mnn * E * (bL / L) ** 4)
    assert 0.05 < factor < 0.95
    assert np.abs(nv @ Xp - factor * A * hinged_mode(bL, s, L)).max() <= 1e-3 * A
    # a bent fiber under a load: the hinged end stays, its curvature vanishes, its tangent turns
    Xb = bent(24, 1.0)
    fE = np.random.default_rng(7).standard_normal((3, 25))
    Xq, _, _, _ = oracle_mod.fiber_step(Xb, np.array([1.0]), 25, eps, E, 5e-3, fE, 12, mu, clamp=[2])
    D = oracle_mod.cheb_diff(24)
    assert np.abs(Xq[:, 24] - Xb[:, 24]).max() <= 1e-10
    assert np.abs(Xq @ (D @ D)[24]).max() <= 1e-8 * np.abs(Xq @ (D @ D)[12]).max() + 1e-10
    assert np.abs((Xq - Xb) @ D[24]).max() > 1e-4


def rot(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def two_fibers(p, L):
    X1 = bent(p, L)
    R = rot([0.2, 1.0, 0.5], 0.7)
    X2 = R @ bent(p, L, amp=-0.2) + np.array([[0.1], [0.35], [0.2]])
    return np.concatenate([X1, X2], axis=1)


def test_rotation_covariance_and_decoupling(oracle_mod):
    p, L, eps, mu, E, dt = 15, 1.0, 0.02, 1.0, 0.8, 5e-3
    n = p + 1
    X = two_fibers(p, L)
    rng = np.random.default_rng(5)
    fE = rng.standard_normal((3, 2 * n))
    Ls = np.array([L, L])
    Xp, T, h, m = oracle_mod.fiber_step(X, Ls, n, eps, E, dt, fE, 60, mu, delta=0.05)
    assert h[-1] <= 1e-11 * h[0]
    R = rot([1.0, -0.4, 0.3], 1.1)
    Xr, Tr, _, _ = oracle_mod.fiber_step(R @ X, Ls, n, eps, E, dt, R @ fE, 60, mu, delta=0.05)
    assert np.abs(Xr - R @ Xp).max() <= 1e-9 * np.abs(Xp).max()
    assert np.abs(Tr - T).max() <= 1e-9 * np.abs(T).max()
    # far apart (1e5 lengths: coupling ~1e-7 of the motion) the fibers move as if alone
    Xf = X.copy()
    Xf[:, n:] += 1e5
    Xpf, Tf, _, _ = oracle_mod.fiber_step(Xf, Ls, n, eps, E, dt, fE, 60, mu)
    for k in range(2):
        sl = slice(k * n, (k + 1) * n)
        Xa, Ta, _, _ = oracle_mod.fiber_step(Xf[:, sl], Ls[:1], n, eps, E, dt, fE[:, sl], 10, mu)
        assert np.abs(Xpf[:, sl] - Xa).max() <= 1e-6 * np.abs(Xa - Xf[:, sl]).max()
        assert np.abs(Tf[sl] - Ta).max() <= 1e-5 * np.abs(Ta).max()
    # close together the coupling matters, and each fiber keeps its length although the
    # other's flow stretches it
    Xn, Tn, _, _ = oracle_mod.fiber_step(X, Ls, n, eps, E, dt, fE, 60, mu)
    X1, _, _, _ = oracle_mod.fiber_step(X[:, :n], Ls[:1], n, eps, E, dt, fE[:, :n], 10, mu)
    assert np.abs(Xn[:, :n] - X1).max() > 1e-3 * np.abs(X1 - X[:, :n]).max()
    Xn, Tn, _, _ = oracle_mod.fiber_step(X, Ls, n, eps, E, 1e-3, fE, 60, mu)
    for k in range(2):      # (without the other fiber's flow in the tension rows: ~2 %)
        sl = slice(k * n, (k + 1) * n)
        assert abs(length(oracle_mod, Xn[:, sl], p) - L) <= 1e-2 * np.abs(Xn[:, sl] - X[:, sl]).max()


def test_gmres_reaches_dense_solution(oracle_mod):
    from oracle.timestep import FiberStep
    p, L, eps, mu, E, dt = 11, 1.0, 0.02, 1.0, 0.8, 5e-3
    n = p + 1
    X = two_fibers(p, L)
    fE = np.random.default_rng(9).standard_normal((3, 2 * n))
    S = FiberStep(X, np.array([L, L]), n, eps, E, dt, mu)
    A = np.stack([S.apply(e) for e in np.eye(8 * n)], axis=1)
    y = np.linalg.solve(A, S.rhs(fE) - A @ np.concatenate([X.ravel(), np.zeros(2 * n)]))
    Xp, T, h, m = oracle_mod.fiber_step(X, np.array([L, L]), n, eps, E, dt, fE, 8 * n, mu)
    assert np.abs(Xp.ravel() - X.ravel() - y[: 6 * n]).max() <= 1e-8 * np.abs(y[: 6 * n]).max()
    assert np.abs(T - y[6 * n:]).max() <= 1e-6 * np.abs(y[6 * n:]).max()
    assert h[30] <= 1e-10 * h[0]      # the block preconditioner leaves only the coupling


# ---- the pins above must catch plausible mistakes in the oracle's time step ----
TS_MUTANTS = {
    "bending_sign": ("return (-self.E * self.per_fiber(self.D4, Xp, 4)", "return (self.E * self.per_fiber(self.D4, Xp, 4)"),
    "bending_scale": ("-self.E * self.per_fiber(self.D4, Xp, 4)", "-self.E * self.per_fiber(self.D4, Xp, 3)"),
    "tension_scale": ("self.per_fiber(self.Da, T[None, :] * self.Xs, 1)", "self.per_fiber(self.Da, T[None, :] * self.Xs, 0)"),
    "tension_sign": ("ten = -(self.tension_local(Xp, T)", "ten = (self.tension_local(Xp, T)"),
    "tension_sss_dropped": ("tf_s = 3.0 * E * (sss3 + ss4) + Tss", "tf_s = 3.0 * E * ss4 + Tss"),
    "tension_curvature_sign": ("ssf = -E * ss4 + k2 * T", "ssf = -E * ss4 - k2 * T"),
    "tension_alpha_as_c": ("return self.c_s * tf + self.c * tf_s - self.alpha * ssf",
                           "return self.c_s * tf + self.c * tf_s - self.c * ssf"),
    "tension_smooth_dropped": ("ten = -(self.tension_local(Xp, T) + self.t_dot_ds(vr))",
                               "ten = -self.tension_local(Xp, T)"),
    "bc_wrong_node": ("s2[:, o], s3[:, o], s2[:, o + p]", "s2[:, o], s3[:, o + 1], s2[:, o + p]"),
    "tension_bc_wrong_node": ("bc_ten[2 * m:2 * m + 2] = [T[o], T[o + p]]", "bc_ten[2 * m:2 * m + 2] = [T[o + 1], T[o + p]]"),
    "rhs_position_dropped": ("pos = self.X / self.dt + v", "pos = v"),
    "resample_points": ("(2.0 * np.arange(m) + 1.0) * np.pi / (2.0 * m)", "(2.0 * np.arange(m) + 0.5) * np.pi / (2.0 * m)"),
    "self_not_excluded": ("excl=oracle.EXCL_SAME_FIBER", "excl=0"),
    "clamp_value_row": ("[s2[:, o], s3[:, o], Xp[:, o + p], second]", "[s2[:, o], s3[:, o], Xp[:, o + p - 1], second]"),
    "clamp_tangent_row": ("second = s1[:, o + p] if self.clamp[m] == 1 else s2[:, o + p]", "second = s2[:, o + p] if self.clamp[m] == 1 else s2[:, o + p]"),
    "hinge_curvature_row": ("second = s1[:, o + p] if self.clamp[m] == 1 else s2[:, o + p]", "second = s1[:, o + p] if self.clamp[m] == 1 else s1[:, o + p]"),
    "clamp_tension_sign": ("bc_ten[2 * m:2 * m + 2] = [T[o], -tv[o + p]]", "bc_ten[2 * m:2 * m + 2] = [T[o], tv[o + p]]"),
    "clamp_tension_local": ("tv = self.c * tf + np.sum(self.tangent * vr, axis=0)", "tv = self.alpha * tf + np.sum(self.tangent * vr, axis=0)"),
    "explicit_dt_velocity": ("pos = Xp / self.dt - self.local_velocity(f)", "pos = Xp / self.dt - 0.5 * self.local_velocity(f)"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(TS_MUTANTS))
def test_timestep_pins_kill_mutant(tmp_path, name):
    import os
    import shutil
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(root, "oracle"), dst, ignore=shutil.ignore_patterns("__pycache__"))
    a, b = TS_MUTANTS[name]
    text = (dst / "timestep.py").read_text()
    assert text.count(a) == 1, f"mutation site for {name} not found once"
    (dst / "timestep.py").write_text(text.replace(a, b))
    code = ("import sys; sys.path.insert(0, %r); import oracle; import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '-m', 'not slow', %r]))"
            % (str(tmp_path), os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
