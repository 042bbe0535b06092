"""GPU mobility solve (device GMRES) and the serving session against the oracle."""
import threading
import time

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


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _oracle_solve(oracle_mod, req, iters=None):
    fs = req["fibers"]
    x, hist, m = oracle_mod.mobility_solve(req["rhs"], fs.xyz, fs.tangent, fs.fiber, fs.length,
                                           fs.nodes_per_fiber, fs.eps, iters or req["iters"])
    return x, hist, m


@pytest.mark.parametrize("n_fib,nodes,iters", [(8, 16, 12), (40, 32, 25), (3, 64, 30), (1, 7, 5)])
def test_mobility_solve_fp64_vs_oracle(S, oracle_mod, n_fib, nodes, iters):
    req = W.serving_request(9, n_fib * 100 + nodes, n_fib=n_fib, nodes=nodes, iters=iters)
    fs = req["fibers"]
    ref, hist, m = _oracle_solve(oracle_mod, req)
    f, res, it = S.mobility_solve(dev(fs.xyz), dev(fs.tangent), dev(fs.length), dev(req["rhs"]),
                                  fs.nodes_per_fiber, fs.eps, iters)
    f = f.cpu().numpy()
    assert it == m
    assert rel(f, ref) <= 1e-10
    assert abs(res - hist[-1]) <= 1e-8 * hist[0] + 1e-6 * hist[-1]


def test_mobility_solve_mixed(S, oracle_mod):
    req = W.serving_request(9, 7, n_fib=60, nodes=32, iters=30)
    fs = req["fibers"]
    ref, hist, m = _oracle_solve(oracle_mod, req)
    f, res, it = S.mobility_solve(dev(fs.xyz), dev(fs.tangent), dev(fs.length), dev(req["rhs"]),
                                  fs.nodes_per_fiber, fs.eps, 30, mixed=True)
    err = rel(f.cpu().numpy(), ref)
    print(f"mixed mobility solve rel err {err:.3e}")
    assert err <= 1e-5


def _submit(sess, req):
    fs = req["fibers"]
    return sess.submit(fs.xyz, fs.tangent, fs.length, req["rhs"], fs.nodes_per_fiber, fs.eps,
                       req["iters"], tag=req["rid"])


def test_session_matches_oracle_and_alone_equals_mix(S, oracle_mod):
    reqs = [W.serving_request(3, rid, n_fib=n, nodes=p, iters=k)
            for rid, (n, p, k) in enumerate([(32, 16, 20), (50, 32, 24), (33, 64, 21), (90, 16, 35),
                                             (40, 32, 22), (64, 16, 28)])]
    alone = []
    with S.Session(hbm_budget_bytes=1 << 30, max_slots=1) as s1:
        for r in reqs:
            alone.append(s1.wait(_submit(s1, r))[0])
    with S.Session(hbm_budget_bytes=1 << 30, max_slots=8) as s8:
        tickets = [_submit(s8, r) for r in reqs]
        mixed = [s8.wait(t) for t in tickets]
    for r, a, (m, st) in zip(reqs, alone, mixed):
        assert np.array_equal(a, m), f"request {r['rid']} differs alone vs in the mix"
        assert st["status"] == 0 and st["iters"] == r["iters"] and st["tag"] == r["rid"]
        assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_finish_ns"]
    for r, a in zip(reqs[:3], alone[:3]):
        ref, _, _ = _oracle_solve(oracle_mod, r)
        assert rel(a, ref) <= 1e-10
    # one-shot solve uses the same kernels and partition: bitwise the same
    r = reqs[1]
    fs = r["fibers"]
    f, _, _ = S.mobility_solve(dev(fs.xyz), dev(fs.tangent), dev(fs.length), dev(r["rhs"]),
                               fs.nodes_per_fiber, fs.eps, r["iters"])
    assert np.array_equal(f.cpu().numpy(), alone[1])


def test_session_mixed_alone_equals_mix(S):
    reqs = [W.serving_request(4, rid, n_fib=n, nodes=p, iters=k)
            for rid, (n, p, k) in enumerate([(40, 32, 20), (70, 16, 25), (33, 64, 22)])]
    with S.Session(hbm_budget_bytes=1 << 30, max_slots=1, mixed=True) as s1:
        alone = [s1.wait(_submit(s1, r))[0] for r in reqs]
    with S.Session(hbm_budget_bytes=1 << 30, max_slots=4, mixed=True) as s4:
        ts = [_submit(s4, r) for r in reqs]
        mix = [s4.wait(t)[0] for t in ts]
    for a, m in zip(alone, mix):
        assert np.array_equal(a, m)


def test_session_mixed_matches_oracle_and_one_shot(S, oracle_mod):
    """Mixed sums in a session: against the oracle's FP64 GMRES (the solve carries the
    sums' 2e-6 error times the operator's conditioning, as the one-shot mixed solve),
    and bitwise equal to the one-shot mixed solve, which runs the same kernels on the
    same partition."""
    reqs = [W.serving_request(4, 100 + rid, n_fib=n, nodes=p, iters=k)
            for rid, (n, p, k) in enumerate([(60, 32, 30), (35, 16, 24), (20, 64, 26)])]
    with S.Session(hbm_budget_bytes=1 << 30, max_slots=4, mixed=True) as s4:
        ts = [_submit(s4, r) for r in reqs]
        out = [s4.wait(t) for t in ts]
    for r, (f, st) in zip(reqs, out):
        ref, _, _ = _oracle_solve(oracle_mod, r)
        err = rel(f, ref)
        print(f"mixed session request {r['rid']}: rel err {err:.3e} after {st['iters']} iterations")
        assert st["status"] == 0
        assert err <= 1e-5
        fs = r["fibers"]
        g, _, _ = S.mobility_solve(dev(fs.xyz), dev(fs.tangent), dev(fs.length), dev(r["rhs"]),
                                   fs.nodes_per_fiber, fs.eps, r["iters"], mixed=True)
        assert np.array_equal(g.cpu().numpy(), f), f"request {r['rid']}: session != one-shot"


@pytest.mark.parametrize("mixed", [False, True])
def test_session_split_matvecs_are_bitwise_unchanged(S, mixed):
    # a pair budget far below one matvec spreads every single-layer sum over
    # many steps; the items write disjoint partials, so nothing changes
    reqs = [W.serving_request(13, rid, n_fib=n, nodes=p, iters=k)
            for rid, (n, p, k) in enumerate([(300, 32, 12), (20, 16, 15), (90, 64, 10)])]
    out = {}
    for sp in (-1, 0, 2_000_000):
        with S.Session(hbm_budget_bytes=1 << 30, max_slots=4, mixed=mixed, step_pairs=sp) as s:
            ts = [_submit(s, r) for r in reqs]
            out[sp] = [s.wait(t) for t in ts]
    # one work item per step (the 320-node request: 20 items per matvec)
    with S.Session(hbm_budget_bytes=1 << 30, max_slots=4, mixed=mixed, step_pairs=1) as s:
        out[1] = [s.wait(_submit(s, reqs[1]))]
    for sp in (0, 2_000_000, 1):
        ref = out[-1] if sp != 1 else out[-1][1:2]
        for (a, sa), (b, sb) in zip(ref, out[sp]):
            assert np.array_equal(a, b), f"step_pairs={sp} changed a result"
            assert sa["iters"] == sb["iters"] and sa["residual"] == sb["residual"]


def test_session_alone_equals_mix_serving_distribution(S):
    # 56 requests drawn like the serving stream (sizes 512 to 131k nodes), submitted
    # in three waves into 64 slots and a 4 GiB budget, against each run alone
    reqs = [W.serving_request(3, 30000 + rid) for rid in range(56)]
    with S.Session(hbm_budget_bytes=4 << 30, max_slots=1, mixed=True) as s1:
        alone = [s1.wait(_submit(s1, r)) for r in reqs]
    with S.Session(hbm_budget_bytes=4 << 30, max_slots=64, mixed=True) as sm:
        ts = []
        for wave in (reqs[:20], reqs[20:40], reqs[40:]):
            ts += [_submit(sm, r) for r in wave]
            time.sleep(0.01)
        mix = [sm.wait(t) for t in ts]
    for r, (a, sa), (m, sm_) in zip(reqs, alone, mix):
        assert np.array_equal(a, m), f"request {r['rid']} differs alone vs in the mix"
        assert sa["iters"] == sm_["iters"] == r["iters"]
        assert np.all(np.isfinite(a))


def test_session_budget_binds_and_errors(S):
    reqs = [W.serving_request(5, rid, n_fib=n, nodes=32, iters=20)
            for rid, n in enumerate([100, 120, 80, 110])]
    foot = [S.solve_footprint(r["fibers"].n_fib, 32, 20) for r in reqs]
    # room for the largest request but not for any two: the budget, not the
    # eight slots, serialises them, in FIFO order
    pair_min = min(a + b for i, a in enumerate(foot) for b in foot[i + 1:])
    budget = (max(foot) + pair_min) // 2
    assert max(foot) < budget < pair_min
    with S.Session(hbm_budget_bytes=budget, max_slots=8) as s:
        ts = [_submit(s, r) for r in reqs]
        out = [s.wait(t) for t in ts]
    stats = [st for _, st in out]
    assert all(st["status"] == 0 for st in stats)
    for a, b in zip(stats, stats[1:]):
        assert b["t_admit_ns"] >= a["t_finish_ns"]
    # the serialised results equal the same requests in a roomy session
    with S.Session(hbm_budget_bytes=1 << 30, max_slots=8) as s:
        ts = [_submit(s, r) for r in reqs]
        roomy = [s.wait(t)[0] for t in ts]
    for (f, _), g in zip(out, roomy):
        assert np.array_equal(f, g)
    # over budget: refused at submit
    with S.Session(hbm_budget_bytes=min(foot) - 1, max_slots=2) as s:
        with pytest.raises(S.StokesError) as ei:
            _submit(s, reqs[0])
        assert ei.value.code == S.E_NOMEM


def test_session_rejects_nonfinite_input(S):
    req = W.serving_request(8, 0, n_fib=10, nodes=16, iters=10)
    with S.Session(hbm_budget_bytes=1 << 28, max_slots=2) as s:
        for field in ("xyz", "tangent", "rhs"):
            bad = dict(req)
            fs = req["fibers"]
            arrs = {"xyz": fs.xyz.copy(), "tangent": fs.tangent.copy(), "rhs": req["rhs"].copy()}
            arrs[field][1, 17] = np.nan if field != "rhs" else np.inf
            with pytest.raises(S.StokesError) as ei:
                s.submit(arrs["xyz"], arrs["tangent"], fs.length, arrs["rhs"],
                         fs.nodes_per_fiber, fs.eps, req["iters"])
            assert ei.value.code == S.E_NONFINITE
            del bad
        fl = req["fibers"].length.copy()
        fl[3] = 0.0
        with pytest.raises(S.StokesError) as ei:
            s.submit(req["fibers"].xyz, req["fibers"].tangent, fl, req["rhs"],
                     req["fibers"].nodes_per_fiber, req["fibers"].eps, req["iters"])
        assert ei.value.code == S.E_INVAL
        # the session still serves a good request afterwards
        f, st = s.wait(_submit(s, req))
        assert st["status"] == 0 and np.all(np.isfinite(f))


def test_session_injected_fault_fails_in_flight_only(S):
    big = W.serving_request(11, 0, n_fib=1500, nodes=32, iters=60)
    small = W.serving_request(11, 1, n_fib=20, nodes=16, iters=10)
    with S.Session(hbm_budget_bytes=1 << 31, max_slots=1) as s:
        ref = s.wait(_submit(s, small))[0]
        t_big = _submit(s, big)
        t_small = _submit(s, small)     # queued behind the big one (one slot)
        time.sleep(0.02)
        s.inject_fault()
        with pytest.raises(S.StokesError) as ei:
            s.wait(t_big)
        assert ei.value.code == S.E_DEVICE
        f, st = s.wait(t_small)         # not in flight at the fault: served normally
        assert st["status"] == 0 and np.array_equal(f, ref)
        f2, st2 = s.wait(_submit(s, small))
        assert st2["status"] == 0 and np.array_equal(f2, ref)


def test_session_second_waiter_gets_busy(S):
    big = W.serving_request(12, 0, n_fib=2000, nodes=64, iters=60)
    with S.Session(hbm_budget_bytes=1 << 32, max_slots=1) as s:
        t = _submit(s, big)
        box = {}

        def waiter():
            box["f"], box["st"] = s.wait(t)

        th = threading.Thread(target=waiter)
        th.start()
        time.sleep(0.05)
        busy = None
        try:
            s.wait(t, timeout_ms=0)
        except S.StokesError as e:
            busy = e.code
        th.join(timeout=120)
        assert box["st"]["status"] == 0
        # the first waiter was still inside wait, or had already taken the result
        assert busy in (S.E_BUSY, S.E_NOTFOUND)


def test_session_cancel_and_destroy_with_pending(S):
    from paper_1602_05650_amd import stokes as SS
    big = W.serving_request(6, 0, n_fib=1500, nodes=32, iters=60)
    small = W.serving_request(6, 1, n_fib=20, nodes=16, iters=10)
    s = S.Session(hbm_budget_bytes=2 << 30, max_slots=1)
    t_big = _submit(s, big)
    t_small = _submit(s, small)        # queued behind the big one (one slot)
    s.cancel(t_small)
    with pytest.raises(SS.StokesError) as ei:
        s.wait(t_small)
    assert ei.value.code == SS.E_CANCELED
    s.cancel(t_big)
    with pytest.raises(SS.StokesError) as ei:
        s.wait(t_big)
    assert ei.value.code == SS.E_CANCELED
    # destroy while a request is pending: a waiting thread gets E_CANCELED
    t3 = _submit(s, big)
    box = {}

    def waiter():
        try:
            s.wait(t3)
            box["rc"] = 0
        except SS.StokesError as e:
            box["rc"] = e.code

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.05)
    s.close()
    th.join(timeout=60)
    assert box.get("rc") in (SS.E_CANCELED, 0)
    # unknown ticket
    with S.Session(hbm_budget_bytes=1 << 24, max_slots=1) as s2:
        with pytest.raises(SS.StokesError) as ei:
            s2.wait(12345)
        assert ei.value.code == SS.E_NOTFOUND


def test_session_timeout(S):
    from paper_1602_05650_amd import stokes as SS
    big = W.serving_request(7, 0, n_fib=2000, nodes=64, iters=60)
    with S.Session(hbm_budget_bytes=4 << 30, max_slots=1) as s:
        t = _submit(s, big)
        with pytest.raises(SS.StokesError) as ei:
            s.wait(t, timeout_ms=1)
        assert ei.value.code == SS.E_TIMEOUT
        f, st = s.wait(t)
        assert st["status"] == 0 and np.all(np.isfinite(f))


@pytest.mark.parametrize("far,mixed,tol", [((6, 0.7), False, 5e-6), ((6, 0.7), True, 2e-5)])
def test_mobility_solve_treecode_far_field_vs_oracle(S, oracle_mod, far, mixed, tol):
    """The other fibers' flow through a treecode plan (the paper's fast summation per
    GMRES matvec) against the oracle's direct FP64 solve: the tree's error on the sum,
    carried through the solve."""
    req = W.serving_request(9, 4000, n_fib=400, nodes=16, iters=25)
    fs = req["fibers"]
    ref, hist, m = _oracle_solve(oracle_mod, req)
    args = (dev(fs.xyz), dev(fs.tangent), dev(fs.length), dev(req["rhs"]), fs.nodes_per_fiber, fs.eps,
            25)
    f_dir, _, _ = S.mobility_solve(*args, mixed=mixed)
    f_far, res, it = S.mobility_solve(*args, mixed=mixed, far=far)
    e_far, e_dir = rel(f_far.cpu().numpy(), ref), rel(f_dir.cpu().numpy(), ref)
    print(f"treecode far field {far} mixed={mixed}: solve vs oracle {e_far:.3e} (direct {e_dir:.3e}), "
          f"{it} iterations")
    assert it == m
    assert e_far <= tol
    # the far field really went through the tree's proxies: the solve differs from the
    # direct one by far more than rounding
    assert rel(f_far.cpu().numpy(), f_dir.cpu().numpy()) > 1e-9


@pytest.mark.parametrize("mixed,tol", [(False, 5e-6), (True, 2e-5)])
def test_session_treecode_requests(S, oracle_mod, mixed, tol):
    """Requests whose u_bar goes through a treecode plan, served beside direct ones: each
    is bitwise equal to the one-shot solve with the same far-field choice (the same
    kernels and the same plan), and the far ones are within the tree's error of the
    oracle's direct FP64 solve."""
    far = (6, 0.7)
    shapes = [(400, 16, 25, True), (60, 32, 18, False), (200, 16, 22, True), (40, 16, 15, False)]
    reqs = [W.serving_request(9, 4000, n_fib=400, nodes=16, iters=25)]   # as the one-shot tree test
    reqs += [W.serving_request(5, 300 + rid, n_fib=n, nodes=p, iters=k)
             for rid, (n, p, k, _) in enumerate(shapes) if rid > 0]
    with S.Session(hbm_budget_bytes=1 << 30, max_slots=4, mixed=mixed) as s:
        ts = []
        for r, sh in zip(reqs, shapes):
            fs = r["fibers"]
            ts.append(s.submit(fs.xyz, fs.tangent, fs.length, r["rhs"], fs.nodes_per_fiber, fs.eps, r["iters"],
                               tag=r["rid"], far=far if sh[3] else None))
        out = [s.wait(t) for t in ts]
    for r, sh, (f, st) in zip(reqs, shapes, out):
        assert st["status"] == 0 and st["iters"] == r["iters"]
        fs = r["fibers"]
        g, _, _ = S.mobility_solve(dev(fs.xyz), dev(fs.tangent), dev(fs.length), dev(r["rhs"]),
                                   fs.nodes_per_fiber, fs.eps, r["iters"], mixed=mixed,
                                   far=far if sh[3] else None)
        assert np.array_equal(g.cpu().numpy(), f), f"request {r['rid']}: session != one-shot"
    ref, _, _ = _oracle_solve(oracle_mod, reqs[0])
    fs = reqs[0]["fibers"]
    d, _, _ = S.mobility_solve(dev(fs.xyz), dev(fs.tangent), dev(fs.length), dev(reqs[0]["rhs"]),
                               fs.nodes_per_fiber, fs.eps, reqs[0]["iters"], mixed=mixed)
    e, e_dir = rel(out[0][0], ref), rel(d.cpu().numpy(), ref)
    diff = rel(out[0][0], d.cpu().numpy())
    print(f"session treecode request (mixed={mixed}, far={far}): rel err vs oracle {e:.3e} "
          f"(direct {e_dir:.3e}; tree vs direct {diff:.3e})")
    assert e <= tol
    assert diff > 1e-9   # the far field really went through the tree's proxies


def test_fiber_step_treecode_far_field(S, oracle_mod):
    """One implicit step with the other fibers' flow through a treecode plan against the
    same step with direct sums (degree 8, theta 0.5: the tree's sum error is ~1e-9)."""
    c = W.config_step(n_fib=300, nodes=16, R=4.0)
    fs = c["fibers"]
    a = (dev(fs.xyz), dev(fs.length), dev(c["f_ext"]), fs.nodes_per_fiber, c["eps"], c["E"], c["dt"])
    X0, T0, r0, i0 = S.fiber_step(*a, iters=40, tol=1e-10)
    X1, T1, r1, i1 = S.fiber_step(*a, iters=40, tol=1e-10, far=(8, 0.5))
    x = fs.xyz
    dX0, dX1 = X0.cpu().numpy() - x, X1.cpu().numpy() - x
    e = np.abs(dX1 - dX0).max() / np.abs(dX0).max()
    print(f"fiber step, treecode far field vs direct: dX {e:.3e}, iterations {i0} / {i1}")
    assert e <= 1e-6
