"""Pins of the oracle's nonlocal slender-body term K_delta (eq. sb-stokes-reg) and of
the fiber block-Jacobi preconditioner (section "Linear solver and preconditioner").

K_delta is checked against the continuous integral, evaluated by adaptive quadrature
(scipy.integrate.quad) on a straight fiber and on a circular arc, where the geometry
and the force are known functions of s; the discrete rule (Clenshaw-Curtis on the CGL
nodes) must converge to it.  Exact properties: zero for a constant force on a straight
fiber, self-adjointness in the quadrature-weighted inner product, translation and
rotation covariance.  The preconditioner is checked by what it must do: on one fiber
it inverts the whole operator (GMRES converges in one iteration), and on several
fibers the preconditioned GMRES reaches the dense solution.
"""
import math

import numpy as np
import pytest

integrate = pytest.importorskip("scipy.integrate")

MU = 0.8


def cgl_s(p, L):
    a = np.cos(np.arange(p + 1) * np.pi / p)
    return 0.5 * L * (1.0 + a)


def force_fn(s):
    return np.array([np.cos(2.0 * s) + 0.3, s * s - 0.5 * s, 1.0 + 0.4 * s ** 3])


def continuous_K(X, T, f, L, delta, s, mu=MU):
    """K_delta[f](s) by adaptive quadrature of the integrand of eq. sb-stokes-reg."""
    c = 1.0 / (8.0 * math.pi * mu)
    xs, ts, fs = X(s), T(s), f(s)
    proj = fs + ts * np.dot(ts, fs)

    def integrand(sp, comp):
        r = xs - X(sp)
        rn = math.sqrt(np.dot(r, r))
        fp = f(sp)
        if rn == 0.0:
            return 0.0
        G = c * (fp / rn + r * np.dot(r, fp) / rn ** 3)
        val = rn / math.sqrt(rn * rn + delta * delta) * G - c * proj / math.sqrt((s - sp) ** 2 + delta * delta)
        return val[comp]

    pts = [s] if 0.0 < s < L else None
    return np.array([integrate.quad(integrand, 0.0, L, args=(c_,), points=pts, limit=400,
                                    epsabs=1e-14, epsrel=1e-13)[0] for c_ in range(3)])


def straight(L, t, x0):
    t = np.asarray(t, float) / np.linalg.norm(t)
    return (lambda s: x0 + s * t), (lambda s: t)


def arc(R, x0):
    X = lambda s: x0 + R * np.array([math.cos(s / R), math.sin(s / R), 0.0])
    T = lambda s: np.array([-math.sin(s / R), math.cos(s / R), 0.0])
    return X, T


def discrete_K(oracle_mod, X, T, L, p, delta, f=force_fn):
    s = cgl_s(p, L)
    xyz = np.stack([X(v) for v in s], axis=1)
    tan = np.stack([T(v) for v in s], axis=1)
    fv = np.stack([f(v) for v in s], axis=1)
    fib = np.zeros(p + 1, dtype=np.int64)
    return s, oracle_mod.nonlocal_sbt(fv, xyz, tan, fib, np.array([L]), p + 1, delta, MU)


@pytest.mark.parametrize("geom", ["straight", "arc"])
def test_nonlocal_converges_to_the_integral(oracle_mod, geom):
    L, delta = 1.3, 0.15
    X, T = straight(L, [1.0, -2.0, 0.5], np.array([0.2, 0.1, -0.3])) if geom == "straight" \
        else arc(0.9, np.array([0.1, 0.0, 0.4]))
    errs = []
    for p in (15, 31, 63):
        s, K = discrete_K(oracle_mod, X, T, L, p, delta)
        ref = np.stack([continuous_K(X, T, force_fn, L, delta, v) for v in s], axis=1)
        errs.append(np.abs(K - ref).max() / np.abs(ref).max())
    # spectral convergence of the smooth integrand (kink width delta, resolved at p >= 31)
    assert errs[1] < errs[0] and errs[2] < 1e-7, errs


def test_nonlocal_constant_force_on_straight_fiber_is_zero(oracle_mod):
    # on a straight fiber |r| = |s - s'| and G(r) f = (I + t t) f / (8 pi mu |r|): the two
    # parts of the integrand are equal term by term for a constant force
    L, p = 2.0, 31
    X, T = straight(L, [0.3, 0.4, -1.0], np.array([1.0, 2.0, 3.0]))
    s, K = discrete_K(oracle_mod, X, T, L, p, 0.01, f=lambda s: np.array([0.7, -1.1, 0.4]))
    assert np.abs(K).max() < 1e-12


def test_nonlocal_uniform_force_on_arc_is_not_zero(oracle_mod):
    # the arc's r-hat differs from its tangent: a constant force gives a nonzero field
    X, T = arc(0.5, np.zeros(3))
    s, K = discrete_K(oracle_mod, X, T, 1.0, 31, 0.05, f=lambda s: np.array([0.0, 1.0, 0.0]))
    assert np.abs(K).max() > 1e-3


def _random_fibers(rng, n_fib, p):
    n = p + 1
    xyz, tan = [], []
    for _ in range(n_fib):
        # a random smooth (cubic) curve, tangents from its derivative
        c = rng.standard_normal((3, 4)) * np.array([1.0, 1.0, 0.3, 0.1])
        a = np.cos(np.arange(n) * np.pi / p)
        pts = c[:, :1] + c[:, 1:2] * a + c[:, 2:3] * a ** 2 + c[:, 3:4] * a ** 3
        d = c[:, 1:2] + 2 * c[:, 2:3] * a + 3 * c[:, 3:4] * a ** 2
        xyz.append(pts)
        tan.append(d / np.linalg.norm(d, axis=0))
    fib = np.repeat(np.arange(n_fib), n)
    return np.concatenate(xyz, axis=1), np.concatenate(tan, axis=1), fib


def test_nonlocal_self_adjoint_in_weighted_inner_product(oracle_mod):
    rng = np.random.default_rng(7)
    p, n_fib = 15, 3
    xyz, tan, fib = _random_fibers(rng, n_fib, p)
    L = rng.uniform(0.5, 2.0, n_fib)
    w = oracle_mod.fiber_quadrature_weights(fib, L, p + 1)
    f, g = rng.standard_normal((2, 3, xyz.shape[1]))
    Kf = oracle_mod.nonlocal_sbt(f, xyz, tan, fib, L, p + 1, 0.05, MU)
    Kg = oracle_mod.nonlocal_sbt(g, xyz, tan, fib, L, p + 1, 0.05, MU)
    a = np.sum(w * np.sum(g * Kf, axis=0))
    b = np.sum(w * np.sum(f * Kg, axis=0))
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def test_nonlocal_translation_rotation_covariance(oracle_mod):
    rng = np.random.default_rng(8)
    p, n_fib = 15, 2
    xyz, tan, fib = _random_fibers(rng, n_fib, p)
    L = np.array([1.0, 1.7])
    f = rng.standard_normal((3, xyz.shape[1]))
    K = oracle_mod.nonlocal_sbt(f, xyz, tan, fib, L, p + 1, 0.02, MU)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    K2 = oracle_mod.nonlocal_sbt(Q @ f, Q @ xyz + 5.0, Q @ tan, fib, L, p + 1, 0.02, MU)
    assert np.abs(K2 - Q @ K).max() <= 1e-12 * np.abs(K).max()


def test_block_preconditioner_inverts_a_lone_fiber(oracle_mod):
    # one fiber: the operator is exactly its self block, so block-preconditioned GMRES
    # is exact after one iteration
    X, T = arc(0.7, np.zeros(3))
    L, p = 1.0, 15
    s = cgl_s(p, L)
    xyz = np.stack([X(v) for v in s], axis=1)
    tan = np.stack([T(v) for v in s], axis=1)
    fib = np.zeros(p + 1, dtype=np.int64)
    rhs = np.random.default_rng(3).standard_normal((3, p + 1))
    x, hist, m = oracle_mod.mobility_solve(rhs, xyz, tan, fib, np.array([L]), p + 1, 0.01, 5,
                                           mu=MU, delta=0.05, precond="block")
    assert hist[1] <= 1e-12 * hist[0]
    Ax = oracle_mod.mobility_apply(x, xyz, tan, fib, np.array([L]), p + 1, 0.01, MU, delta=0.05)
    assert np.abs(Ax - rhs).max() <= 1e-11 * np.abs(rhs).max()
    # the local preconditioner needs more than one iteration on the same problem
    _, hist_l, _ = oracle_mod.mobility_solve(rhs, xyz, tan, fib, np.array([L]), p + 1, 0.01, 5,
                                             mu=MU, delta=0.05, precond="local")
    assert hist_l[1] > 1e-6 * hist_l[0]


def test_nonlocal_block_gmres_matches_dense_solve(oracle_mod):
    rng = np.random.default_rng(9)
    p, n_fib = 7, 4
    xyz, tan, fib = _random_fibers(rng, n_fib, p)
    xyz = xyz + np.repeat(rng.uniform(-3, 3, (3, n_fib)), p + 1, axis=1)
    L = rng.uniform(0.8, 1.5, n_fib)
    n = xyz.shape[1]
    args = (xyz, tan, fib, L, p + 1, 0.01)

    def A(v):
        return oracle_mod.mobility_apply(v.reshape(3, n), *args, MU, delta=0.03).ravel()

    dense = np.stack([A(e) for e in np.eye(3 * n)], axis=1)
    rhs = rng.standard_normal((3, n))
    ref = np.linalg.solve(dense, rhs.ravel()).reshape(3, n)
    x, hist, m = oracle_mod.mobility_solve(rhs, *args, 3 * n, mu=MU, delta=0.03, precond="block")
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    # the nonlocal term changes the solution (how much depends on how rough the
    # force is: for node-to-node noise its diagonal part nearly cancels M)
    xl, _, _ = oracle_mod.mobility_solve(rhs, *args, 3 * n, mu=MU)
    assert np.linalg.norm(x - xl) > 1e-4 * np.linalg.norm(xl)


# ---- the pins above must catch plausible mistakes in the oracle's nonlocal code ----
PY_MUTANTS = {
    "rr_term_dropped": ("G_fk = c * (f[:, ks] / rn + r * (rf / rn ** 3))", "G_fk = c * (f[:, ks] / rn)"),
    "phi_dropped": ("phi = rn / np.sqrt(rn * rn + delta * delta)", "phi = 1.0"),
    "psi_wrong_delta": ("psi = 1.0 / np.sqrt((s[i] - s[ks]) ** 2 + delta * delta)",
                        "psi = 1.0 / np.sqrt((s[i] - s[ks]) ** 2 + 4.0 * delta * delta)"),
    "second_term_uses_f_k": ("- c * proj_fi[:, None] * psi", "- c * f[:, ks] * psi"),
    "tt_projection_dropped": ("proj_fi = f[:, i] + ti * np.dot(ti, f[:, i])", "proj_fi = f[:, i]"),
    "target_weight": ("np.sum(w[ks] * (phi * G_fk", "np.sum(w[i] * (phi * G_fk"),
    "block_column_layout": ("            e.flat[col] = 1.0", "            e.T.flat[col] = 1.0"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_nonlocal_pins_kill_mutant(tmp_path, name):
    import os
    import shutil
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = os.path.join(root, "oracle")
    dst = tmp_path / "oracle"
    shutil.copytree(src, dst, ignore=shutil.ignore_patterns("__pycache__"))
    a, b = PY_MUTANTS[name]
    text = (dst / "__init__.py").read_text()
    assert text.count(a) == 1, f"mutation site for {name} not found once"
    (dst / "__init__.py").write_text(text.replace(a, b))
    # import the mutated copy first, so the pins' `import oracle` finds it
    code = ("import sys; sys.path.insert(0, %r); import oracle; import pytest; "
            "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '-m', 'not slow', %r]))"
            % (str(tmp_path), os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
