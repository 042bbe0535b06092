"""GPU implicit fiber time step (stokes_fiber_step) against the oracle and closed forms.

Parity: the same seeded bent fibers and forces on both sides, the same number of
GMRES iterations; X+ - X and T+ element by element.  The step's operator holds up to
the fourth derivative of the nodes in both row blocks, so rounding of the node values
is amplified by up to ~p^8 and the tolerance grows with the nodes per fiber: X+ - X
and T+ to 2e-9 of their size at 16 nodes, scaled by (n/16)^8 (measured: 0.03-0.09 of
that bound with several fibers, 0.23 for the single 20-node fiber).  At the full benchmark size the GPU solution is checked by the
oracle's own residual of the discrete system.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1602_05650_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05650_amd import stokes
    return stokes


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def small_case(seed, n_fib, nodes, R=1.0, amp=0.8, eps=0.02):
    g = np.random.default_rng(seed)
    fs = W.bent_fibers(g, n_fib, nodes, R, L=1.0, eps=eps, amp=amp, gap=0.1)
    f = np.random.default_rng(seed + 100).standard_normal((3, fs.n))
    return fs, f


def tolerances(n):
    t = 2e-9 * max(1.0, (n / 16) ** 8)
    return t, t


@pytest.mark.parametrize("n_fib,nodes,delta,E,dt,seed", [
    (4, 16, None, 1.0, 2e-3, 1),
    (4, 16, 0.05, 1.0, 2e-3, 2),
    (3, 6, None, 0.5, 5e-3, 3),        # fewest nodes the collocation allows
    (5, 31, None, 1.0, 3e-3, 4),       # the paper's 31 points per fiber
    (2, 32, 0.05, 2.0, 1e-3, 5),
    (2, 48, None, 1.0, 1e-3, 6),       # most nodes (4 n <= 192 per block)
    (1, 20, None, 1.0, 2e-3, 7),       # a single fiber: no other fibers' flow
    (3, 16, None, 0.0, 2e-3, 8),       # no bending stiffness
])
def test_step_parity_with_oracle(S, oracle_mod, n_fib, nodes, delta, E, dt, seed):
    fs, f = small_case(seed, n_fib, nodes)
    iters = min(4 * nodes * n_fib, 30)
    eps, mu = fs.eps, 0.9
    print(f"case n_fib={n_fib} nodes={nodes} delta={delta} E={E}", flush=True)
    Xo, To, h, m = oracle_mod.fiber_step(fs.xyz, fs.length, nodes, eps, E, dt, f, iters, mu,
                                         delta=delta)
    Xg, Tg, res, it = S.fiber_step(dev(fs.xyz), dev(fs.length), dev(f), nodes, eps, E, dt, mu=mu,
                                   delta=delta, iters=iters)
    Xg, Tg = Xg.cpu().numpy(), Tg.cpu().numpy()
    dXo, dXg = Xo - fs.xyz, Xg - fs.xyz
    ex = np.abs(dXg - dXo).max() / np.abs(dXo).max()
    eT = np.abs(Tg - To).max() / max(np.abs(To).max(), 1e-300)
    tx, tT = tolerances(nodes)
    print(f"  dX err {ex:.2e} (tol {tx:.1e}), T err {eT:.2e} (tol {tT:.1e}), iters {it}/{m}, "
          f"resid {res:.3e} vs {h[-1]:.3e} of {h[0]:.3e}")
    assert it == m
    assert abs(res - h[-1]) <= 1e-6 * h[0] + 1e-3 * h[-1]
    assert ex <= tx
    assert eT <= tT


@pytest.mark.parametrize("n_fib,nodes,delta,seed", [(4, 16, None, 41), (3, 32, None, 42), (3, 20, 0.05, 43),
                                                 (2, 40, None, 44)])
def test_attached_step_parity_with_oracle(S, oracle_mod, n_fib, nodes, delta, seed):
    # minus ends clamped (1) or hinged (2) to a body at rest on some fibers, free (0) on
    # the others (every block path: built in place, from the prepared products, the wide
    # kernel)
    fs, f = small_case(seed, n_fib, nodes)
    clamp = (np.arange(n_fib) + 1) % 3
    E, dt, mu, iters = 1.0, 2e-3, 0.9, 30
    print(f"attached case n_fib={n_fib} nodes={nodes} delta={delta} ends={clamp.tolist()}", flush=True)
    Xo, To, h, m = oracle_mod.fiber_step(fs.xyz, fs.length, nodes, fs.eps, E, dt, f, iters, mu,
                                         delta=delta, clamp=clamp)
    Xg, Tg, res, it = S.fiber_step(dev(fs.xyz), dev(fs.length), dev(f), nodes, fs.eps, E, dt, mu=mu,
                                   delta=delta, iters=iters, clamp=clamp)
    Xg, Tg = Xg.cpu().numpy(), Tg.cpu().numpy()
    dXo = Xo - fs.xyz
    ex = np.abs(Xg - Xo).max() / np.abs(dXo).max()
    eT = np.abs(Tg - To).max() / np.abs(To).max()
    tx, tT = tolerances(nodes)
    print(f"  dX err {ex:.2e} (tol {tx:.1e}), T err {eT:.2e}, iters {it}/{m}")
    assert it == m and ex <= tx and eT <= tT
    for k in np.flatnonzero(clamp):         # the attached ends stay where they were
        e = (k + 1) * nodes - 1
        assert np.abs(Xg[:, e] - fs.xyz[:, e]).max() <= 1e-12 * (1 + np.abs(fs.xyz).max())


def test_end_condition_values_checked(S):
    fs, f = small_case(3, 2, 16)
    with pytest.raises(ValueError):
        S.fiber_step(dev(fs.xyz), dev(fs.length), dev(f), 16, fs.eps, 1.0, 1e-3, clamp=[0, 3])


@pytest.mark.parametrize("kind", [1, 2])
def test_attached_straight_fiber_holds_a_tangential_load(S, kind):
    # clamped or hinged: a straight fiber stays straight, so both hold the load alike
    n, L, eps, mu, E, dt = 21, 1.4, 0.02, 0.8, 1.3, 2e-3
    a = np.cos(np.arange(n) * np.pi / (n - 1))
    t = np.array([0.5, -1.0, 0.3])
    t /= np.linalg.norm(t)
    X = np.array([0.1, 0.0, 0.2])[:, None] + 0.5 * L * a[None, :] * t[:, None]
    s = 0.5 * L * (1 + a)
    g = s ** 2 - 0.3 * s + 0.2
    G = lambda x: x ** 3 / 3 - 0.15 * x ** 2 + 0.2 * x
    Xg, Tg, res, it = S.fiber_step(dev(X), dev([L]), dev(g[None, :] * t[:, None]), n, eps, E, dt, mu=mu,
                                   iters=8, clamp=[kind])
    ref = G(L) - G(s)
    assert np.abs(Tg.cpu().numpy() - ref).max() <= 1e-8 * np.abs(ref).max()
    assert np.abs(Xg.cpu().numpy() - X).max() <= 1e-10


def test_step_mixed_precision_sums(S, oracle_mod):
    fs, f = small_case(11, 6, 16)
    E, dt, mu = 1.0, 2e-3, 1.0
    Xo, To, h, m = oracle_mod.fiber_step(fs.xyz, fs.length, 16, fs.eps, E, dt, f, 30, mu)
    Xg, Tg, res, it = S.fiber_step(dev(fs.xyz), dev(fs.length), dev(f), 16, fs.eps, E, dt, mu=mu,
                                   iters=30, mixed=True, near_r=0.3)
    dXo = Xo - fs.xyz
    ex = np.abs(Xg.cpu().numpy() - Xo).max() / np.abs(dXo).max()
    eT = np.abs(Tg.cpu().numpy() - To).max() / np.abs(To).max()
    print(f"mixed: dX err {ex:.2e}, T err {eT:.2e}")
    assert ex <= 2e-5 and eT <= 2e-4


def test_straight_fiber_translates_and_beam_mode_decays(S):
    # uniform force on a straight fiber: rigid translation with M f, no tension
    n, L, eps, mu, E, dt = 24, 1.3, 0.01, 0.7, 2.0, 1e-3
    a = np.cos(np.arange(n) * np.pi / (n - 1))
    t = np.array([0.3, -0.4, 0.866])
    t /= np.linalg.norm(t)
    X = np.array([0.2, 0.1, -0.3])[:, None] + 0.5 * L * a[None, :] * t[:, None]
    fv = np.array([0.4, -1.1, 0.25])
    kap = -math.log(eps * eps * math.e)
    U = ((kap + 2) * fv + (kap - 2) * t * np.dot(t, fv)) / (8 * math.pi * mu)
    Xg, Tg, res, it = S.fiber_step(dev(X), dev([L]), dev(np.repeat(fv[:, None], n, 1)), n, eps, E, dt,
                                   mu=mu, iters=8)
    assert np.abs(Xg.cpu().numpy() - X - dt * U[:, None]).max() <= 1e-6 * dt * np.abs(U).max()
    assert np.abs(Tg.cpu().numpy()).max() <= 1e-4 * np.abs(fv).max() * L
    # a free-free beam mode relaxes by 1/(1 + dt M_nn E b^4)
    bL, A, n, L, E, dt = 4.730040744862704, 1e-6, 32, 1.2, 1.5, 2e-3
    a = np.cos(np.arange(n) * np.pi / (n - 1))
    s = 0.5 * L * (1 + a)
    b = bL / L
    sig = (math.cosh(bL) - math.cos(bL)) / (math.sinh(bL) - math.sin(bL))
    phi = np.cosh(b * s) + np.cos(b * s) - sig * (np.sinh(b * s) + np.sin(b * s))
    nv = np.cross(t, [0.3, 1.0, -0.2])
    nv /= np.linalg.norm(nv)
    X = (s - 0.5 * L)[None, :] * t[:, None] + A * phi[None, :] * nv[:, None]
    Xg, Tg, res, it = S.fiber_step(dev(X), dev([L]), dev(np.zeros((3, n))), n, eps, E, dt, mu=mu,
                                   iters=8)
    fac = 1.0 / (1.0 + dt * (kap + 2) / (8 * math.pi * mu) * E * b ** 4)
    assert np.abs(nv @ Xg.cpu().numpy() - fac * A * phi).max() <= 1e-4 * A


@pytest.mark.parametrize("nodes,delta,clamp", [(6, None, False), (16, None, False), (31, None, False),
                                               (32, None, False), (32, 0.05, False), (20, 0.05, False),
                                               (40, None, False), (48, 0.05, False), (32, None, 1),
                                               (20, 0.05, 1), (40, None, 1), (32, None, 2), (20, 0.05, 2),
                                               (40, None, 2)])
def test_single_fiber_block_is_the_inverse(S, oracle_mod, nodes, delta, clamp):
    # one fiber: the block-Jacobi preconditioner is the exact inverse of the operator, so
    # one GMRES iteration leaves only rounding amplified by the block's conditioning
    # (~p^8 after row equilibration; a wrong inverse leaves O(1)).  With the nonlocal
    # term the block's columns carry D4 (entries ~p^8) through a sum over the fiber's
    # nodes, which costs another ~eps p^8 of accuracy in forming it (a preconditioner
    # only: the solution is the operator's).  Every block path: built in place for
    # <= 32 nodes, from the prepared products with the nonlocal term, the wide kernel
    # above 32.
    from oracle.timestep import FiberStep
    fs, f = small_case(21 + nodes, 1, nodes)
    E, dt = 1.0, 2e-3
    St = FiberStep(fs.xyz, fs.length, nodes, fs.eps, E, dt, 1.0, delta=delta, clamp=[clamp])
    beta = np.linalg.norm(St.rhs(f) - St.apply(np.concatenate([fs.xyz.ravel(), np.zeros(nodes)])))
    X1, T1, res, it = S.fiber_step(dev(fs.xyz), dev(fs.length), dev(f), nodes, fs.eps, E, dt,
                                   delta=delta, iters=1, clamp=[int(clamp)])
    # (an attached end puts unit position rows beside the D_s^4 rows: a little worse again)
    cap = 0.2 if delta else (1e-2 if clamp else 1e-3)
    bound = min(cap, 1e-6 * max(1.0, (nodes / 16) ** 8) * (100.0 if delta else (10.0 if clamp else 1.0)))
    print(f"nodes {nodes} delta {delta} clamp {clamp}: residual after one iteration {res / beta:.2e} "
          f"(bound {bound:.1e})")
    assert it == 1 and res / beta <= bound


def test_buffers_reused_across_calls(S):
    # the step keeps its device buffer per stream: calls of other sizes in between, and a
    # release of every workspace, leave the result of the same input bitwise unchanged
    fs1, f1 = small_case(31, 4, 16)
    fs2, f2 = small_case(32, 3, 32)

    def run(fs, f, n):
        X, T, res, it = S.fiber_step(dev(fs.xyz), dev(fs.length), dev(f), n, fs.eps, 1.0, 2e-3, iters=12)
        return X.cpu().numpy(), T.cpu().numpy()
    a = run(fs1, f1, 16)
    run(fs2, f2, 32)             # larger: the buffer grows, the tables change
    b = run(fs1, f1, 16)
    S.release_workspace()
    c = run(fs1, f1, 16)
    for u in (b, c):
        assert np.array_equal(u[0], a[0]) and np.array_equal(u[1], a[1])


def test_step_on_a_caller_stream_matches_the_default_stream(S):
    # the blocks are formed on a library side stream forked from and joined back into the
    # caller's stream: on a stream of the caller's own, also with calls of another size
    # in between and the caller's stream busy with other work, the result is bitwise the
    # default stream's
    import torch
    fs1, f1 = small_case(33, 5, 24)
    fs2, f2 = small_case(34, 2, 40)
    args1 = (dev(fs1.xyz), dev(fs1.length), dev(f1), 24, fs1.eps, 1.0, 2e-3)
    ref = S.fiber_step(*args1, iters=12)
    ref = (ref[0].cpu().numpy(), ref[1].cpu().numpy())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())   # (the inputs were copied on the default stream)
    with torch.cuda.stream(side):
        busy = torch.randn(2048, 2048, dtype=torch.float64, device="cuda")
        for _ in range(3):
            busy = busy @ busy.T.contiguous() / 2048.0   # work queued ahead of the step
        outs = []
        for _ in range(2):
            X, T, res, it = S.fiber_step(*args1, iters=12, stream=side)
            outs.append((X.cpu().numpy(), T.cpu().numpy()))
            S.fiber_step(dev(fs2.xyz), dev(fs2.length), dev(f2), 40, fs2.eps, 1.0, 2e-3, iters=4,
                         stream=side)
    torch.cuda.synchronize()
    for X, T in outs:
        assert np.array_equal(X, ref[0]) and np.array_equal(T, ref[1])


def test_fiber_at_rest_stays(S):
    # a straight fiber without force: the right-hand side is rounding (D4 of a line,
    # ~eps p^8 (2/L)^4 E dt |M| |X| ~ 1e-11 here), the fiber stays where it is and carries
    # no tension
    n, L = 16, 1.0
    a = np.cos(np.arange(n) * np.pi / (n - 1))
    X = np.stack([0.5 * L * a, 0.2 + 0 * a, 0 * a])
    Xg, Tg, res, it = S.fiber_step(dev(X), dev([L]), dev(np.zeros((3, n))), n, 0.01, 1.0, 1e-3,
                                   iters=5)
    assert np.abs(Xg.cpu().numpy() - X).max() <= 1e-10
    assert np.abs(Tg.cpu().numpy()).max() <= 1e-8


def test_full_size_step_solves_the_oracle_system(S, oracle_mod):
    """2048 free fibers x 32 nodes (the benchmark step): the oracle evaluates its own
    residual of the discrete system at the GPU's solution, which must sit at the
    rounding floor of that system in FP64.  Two floors: applying the operator (entries
    up to ~p^8 / dt against node values), measured as the change of the oracle's A y
    when y is scaled by 1 + 2^-40 (minus the exact linear change); and the right-hand
    side (D1 of the bending velocity of the current nodes, ~p^10), measured as the
    change of the oracle's b under a rigid translation of all fibers, which leaves the
    exact system unchanged."""
    from oracle.timestep import FiberStep
    c = W.config_step()
    fs = c["fibers"]
    n = fs.nodes_per_fiber
    print("full-size step: 2048 x 32", flush=True)
    Xg, Tg, res, it = S.fiber_step(dev(fs.xyz), dev(fs.length), dev(c["f_ext"]), n, c["eps"], c["E"],
                                   c["dt"], mu=c["mu"], iters=30)
    Xg, Tg = Xg.cpu().numpy(), Tg.cpu().numpy()
    N = fs.n

    def system(X):
        St = FiberStep(X, fs.length, n, c["eps"], c["E"], c["dt"], c["mu"], nthreads=16)
        return St, St.rhs(c["f_ext"]) - St.apply(np.concatenate([X.ravel(), np.zeros(N)]))

    St, b = system(fs.xyz)
    y = np.concatenate([(Xg - fs.xyz).ravel(), Tg])
    Ay = St.apply(y)
    d = 2.0 ** -40
    floor_a = np.linalg.norm(St.apply(y * (1 + d)) - (1 + d) * Ay)
    floor_b = np.linalg.norm(system(fs.xyz + np.array([[1 / 3], [-0.7], [0.55]]))[1] - b)
    r = np.linalg.norm(Ay - b)
    beta = np.linalg.norm(b)
    print(f"  iters {it}, GPU residual {res / beta:.3e}, oracle residual {r / beta:.3e}, "
          f"floors: operator {floor_a / beta:.3e}, right-hand side {floor_b / beta:.3e}")
    assert res / beta <= 1e-6
    assert r <= 3 * (floor_a + floor_b) + 1e-6 * beta
    # a wrong solution is far from it: the tension dropped
    y0 = y.copy()
    y0[3 * N:] = 0.0
    assert np.linalg.norm(St.apply(y0) - b) > 100 * max(r, floor_a + floor_b)
