"""GPU parity of the kernel sums against the CPU oracle, through the C ABI.

FP64 path: relative L2 error <= 1e-12 against the FP64 oracle.
Mixed path: relative max-norm error ||e||_inf / ||u||_inf <= 2e-6.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1602_05650_amd import workloads as W  # noqa: E402

FP64_TOL = 1e-12
MIXED_TOL = 2e-6
NTHREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_05650_amd import stokes
    return stokes


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def rel_max(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _random_fibers(seed, n, n_trg_extra=0):
    """n nodes in fibers of 7 (last one ragged), random positions, weights, lengths."""
    rng = np.random.default_rng(seed)
    n_fib = max(1, (n + 6) // 7)
    fib = np.minimum(np.arange(n) // 7, n_fib - 1).astype(np.int32)
    xyz = W.uniform_ball(rng, n, 1.5).T.copy()
    f = rng.standard_normal((3, n))
    w = rng.uniform(0.5, 1.5, n)
    L = rng.uniform(0.5, 2.0, n_fib)
    trg = W.uniform_ball(rng, n_trg_extra, 1.5).T.copy()
    tself = rng.integers(-1, n, n_trg_extra).astype(np.int64)
    tfib = rng.integers(-1, n_fib, n_trg_extra).astype(np.int32)
    return dict(xyz=xyz, f=f, w=w, fib=fib, L=L, trg=trg, tself=tself, tfib=tfib)


EXCL_ORACLE = {"self": 1, "fiber": 2, None: 0}


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 63, 64, 65, 257, 1000])
@pytest.mark.parametrize("excl", ["self", "fiber", None])
def test_sl_random_shapes_targets_are_sources(S, oracle_mod, n, excl):
    g = _random_fibers(n * 7 + len(str(excl)), n)
    eps = 0.02
    ref = oracle_mod.sl(g["xyz"], g["f"], src_weight=g["w"], src_fiber=g["fib"], fiber_len=g["L"],
                        eps=eps, mu=0.8, excl=EXCL_ORACLE[excl], doublet=True)
    args = dict(src_weight=dev(g["w"]), src_fiber=dev(g["fib"], torch.int32), fiber_len=dev(g["L"]),
                eps=eps, mu=0.8, excl=excl)
    u64 = host(S.sl_eval(dev(g["xyz"]), dev(g["f"]), **args))
    u32 = host(S.sl_eval(dev(g["xyz"]), dev(g["f"]), mixed=True, near_r=0.05, **args))
    if np.abs(ref).max() == 0:
        assert np.abs(u64).max() == 0 and np.abs(u32).max() == 0
        return
    assert rel_l2(u64, ref) <= FP64_TOL
    assert rel_max(u32, ref) <= MIXED_TOL


@pytest.mark.parametrize("n", [1, 33, 257, 1000])
@pytest.mark.parametrize("excl", ["self", "fiber", None])
@pytest.mark.parametrize("doublet", [True, False])
def test_sl_explicit_targets(S, oracle_mod, n, excl, doublet):
    g = _random_fibers(n + 3, n, n_trg_extra=n + 17)
    eps = 0.03
    kw = dict(src_weight=g["w"], src_fiber=g["fib"], fiber_len=g["L"], eps=eps, trg_xyz=g["trg"],
              excl=EXCL_ORACLE[excl], doublet=doublet)
    if excl == "self":
        kw["trg_self"] = g["tself"]
    if excl == "fiber":
        kw["trg_fiber"] = g["tfib"]
    ref = oracle_mod.sl(g["xyz"], g["f"], **kw)
    dargs = dict(src_weight=dev(g["w"]), src_fiber=dev(g["fib"], torch.int32),
                 fiber_len=dev(g["L"]), eps=eps, trg_xyz=dev(g["trg"]), excl=excl, doublet=doublet)
    if excl == "self":
        dargs["trg_self"] = dev(g["tself"], torch.int64)
    if excl == "fiber":
        dargs["trg_fiber"] = dev(g["tfib"], torch.int32)
    u64 = host(S.sl_eval(dev(g["xyz"]), dev(g["f"]), **dargs))
    u32 = host(S.sl_eval(dev(g["xyz"]), dev(g["f"]), mixed=True, near_r=0.05, **dargs))
    assert rel_l2(u64, ref) <= FP64_TOL
    assert rel_max(u32, ref) <= MIXED_TOL


def test_sl_config0(S, oracle_mod):
    c = W.config0()
    fs = c["fibers"]
    ref = oracle_mod.sl(fs.xyz, c["force"], src_fiber=fs.fiber, fiber_len=fs.length, eps=fs.eps,
                        excl=1)
    a = dict(src_fiber=dev(fs.fiber, torch.int32), fiber_len=dev(fs.length), eps=fs.eps)
    u64, d64 = S.sl_eval(dev(fs.xyz), dev(c["force"]), diag=True, **a)
    u32, d32 = S.sl_eval(dev(fs.xyz), dev(c["force"]), mixed=True, diag=True, **a)
    assert rel_l2(host(u64), ref) <= FP64_TOL
    assert rel_max(host(u32), ref) <= MIXED_TOL
    assert d64.pairs == 512 * 511 and d32.pairs == 512 * 511
    assert d64.coincident == 0 and d64.near_pairs == 0 and d32.near_pairs > 0


@pytest.fixture(scope="module")
def cfg1():
    return W.config1()


def _cfg1_targets(c):
    fs, sph = c["fibers"], c["sphere"]
    trg = np.concatenate([fs.xyz, sph.xyz], axis=1)
    sl_self = np.concatenate([np.arange(fs.n), -np.ones(sph.n, dtype=np.int64)])
    dl_self = np.concatenate([-np.ones(fs.n, dtype=np.int64), np.arange(sph.n)])
    return trg, sl_self, dl_self


@pytest.fixture(scope="module")
def cfg1_ref(cfg1, oracle_mod):
    c = cfg1
    fs, sph = c["fibers"], c["sphere"]
    trg, sl_self, dl_self = _cfg1_targets(c)
    u_sl = oracle_mod.sl(fs.xyz, c["force"], src_fiber=fs.fiber, fiber_len=fs.length, eps=fs.eps,
                         trg_xyz=trg, trg_self=sl_self, excl=1, nthreads=NTHREADS)
    u_dl = oracle_mod.dl(sph.xyz, sph.normal, sph.weight, c["q"], trg_xyz=trg, trg_self=dl_self,
                         subtract=True, nthreads=NTHREADS)
    return u_sl, u_dl


def _cfg1_gpu(S, c, mixed, near_sl=0.0, near_dl=0.0):
    fs, sph = c["fibers"], c["sphere"]
    trg, sl_self, dl_self = _cfg1_targets(c)
    u_sl = S.sl_eval(dev(fs.xyz), dev(c["force"]), src_fiber=dev(fs.fiber, torch.int32),
                     fiber_len=dev(fs.length), eps=fs.eps, trg_xyz=dev(trg),
                     trg_self=dev(sl_self, torch.int64), mixed=mixed, near_r=near_sl)
    u_dl = S.dl_eval(dev(sph.xyz), dev(sph.normal), dev(sph.weight), dev(c["q"]), trg_xyz=dev(trg),
                     trg_self=dev(dl_self, torch.int64), mixed=mixed, near_r=near_dl)
    return host(u_sl), host(u_dl)


def test_config1_fp64(S, cfg1, cfg1_ref):
    u_sl, u_dl = _cfg1_gpu(S, cfg1, False)
    assert rel_l2(u_sl, cfg1_ref[0]) <= FP64_TOL
    assert rel_l2(u_dl, cfg1_ref[1]) <= FP64_TOL


def test_config1_mixed(S, cfg1, cfg1_ref):
    """The radii the benchmark times: near_r 0 selects two fiber radii (single layer) and
    0.02 (double layer).  Each sum is gated on its own over all 38,912 targets."""
    u_sl, u_dl = _cfg1_gpu(S, cfg1, True)
    e_sl, e_dl = rel_max(u_sl, cfg1_ref[0]), rel_max(u_dl, cfg1_ref[1])
    print(f"config1 mixed (default radii): SL rel max {e_sl:.3e}, DL rel max {e_dl:.3e}")
    assert e_sl <= MIXED_TOL
    assert e_dl <= MIXED_TOL


def test_config1_mixed_wide_near_radius(S, cfg1, cfg1_ref):
    """Wider FP64 radii only move pairs to FP64: the bound still holds."""
    u_sl, u_dl = _cfg1_gpu(S, cfg1, True, near_sl=0.06, near_dl=0.3)
    assert rel_max(u_sl, cfg1_ref[0]) <= MIXED_TOL
    assert rel_max(u_dl, cfg1_ref[1]) <= MIXED_TOL


def test_config1_mixed_sphere_targets_alone(S, cfg1, cfg1_ref):
    """The double layer at the sphere's own points alone (the principal value of a random
    density, whose cancellation leaves |u| ~ 0.08 |q|): the hardest case for FP32 pairs."""
    n_f = cfg1["fibers"].n
    _, u_dl = _cfg1_gpu(S, cfg1, True)
    e = rel_max(u_dl[:, n_f:], cfg1_ref[1][:, n_f:])
    print(f"config1 mixed DL, sphere targets only: rel max {e:.3e}")
    assert e <= MIXED_TOL


def test_determinism(S, cfg1):
    a = _cfg1_gpu(S, cfg1, True)
    b = _cfg1_gpu(S, cfg1, True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    c = _cfg1_gpu(S, cfg1, False)
    d = _cfg1_gpu(S, cfg1, False)
    assert np.array_equal(c[0], d[0]) and np.array_equal(c[1], d[1])


def test_sharded_equals_unsharded(S, cfg1):
    """Targets split into 4 shards (the per-GPU share of a target-sharded run)."""
    c = cfg1
    fs = c["fibers"]
    full = host(S.sl_eval(dev(fs.xyz), dev(c["force"]), src_fiber=dev(fs.fiber, torch.int32),
                          fiber_len=dev(fs.length), eps=fs.eps))
    parts = []
    for idx in np.array_split(np.arange(fs.n), 4):
        parts.append(host(S.sl_eval(dev(fs.xyz), dev(c["force"]),
                                    src_fiber=dev(fs.fiber, torch.int32), fiber_len=dev(fs.length),
                                    eps=fs.eps, trg_xyz=dev(fs.xyz[:, idx]),
                                    trg_self=dev(idx.astype(np.int64), torch.int64))))
    sharded = np.concatenate(parts, axis=1)
    assert rel_l2(sharded, full) <= 1e-14


def test_dl_identities_gpu(S):
    sph = W.sphere_surface(32, 48, 1.7)
    q0 = np.array([0.5, -1.5, 2.0])
    q = np.repeat(q0[:, None], sph.n, axis=1)
    rng = np.random.default_rng(3)
    inside = W.uniform_ball(rng, 10, 1.0).T.copy()
    outside = (W.uniform_sphere_dirs(rng, 10) * 3.0).T.copy()
    args = (dev(sph.xyz), dev(sph.normal), dev(sph.weight), dev(q))
    for mixed in (False, True):
        tol = 1e-11 if not mixed else 1e-5
        u_in = host(S.dl_eval(*args, trg_xyz=dev(inside), mixed=mixed))
        u_out = host(S.dl_eval(*args, trg_xyz=dev(outside), mixed=mixed))
        u_on = host(S.dl_eval(*args, mixed=mixed))
        np.testing.assert_allclose(u_in, -np.repeat(q0[:, None], 10, axis=1), atol=tol * 2)
        np.testing.assert_allclose(u_out, 0.0, atol=max(tol * 2, 1e-10))  # quadrature error off S
        np.testing.assert_allclose(u_on, -0.5 * q, atol=tol * 2)


@pytest.mark.parametrize("subtract", [True, False])
@pytest.mark.parametrize("near_r", [0.0, 0.3])
def test_dl_random_parity(S, oracle_mod, subtract, near_r):
    rng = np.random.default_rng(17)
    sph = W.sphere_surface(16, 24, 1.0)
    q = rng.standard_normal((3, sph.n))
    trg = np.concatenate([sph.xyz, W.uniform_ball(rng, 77, 1.4).T], axis=1)
    tself = np.concatenate([np.arange(sph.n), -np.ones(77, dtype=np.int64)])
    ref = oracle_mod.dl(sph.xyz, sph.normal, sph.weight, q, trg_xyz=trg, trg_self=tself,
                        subtract=subtract)
    args = (dev(sph.xyz), dev(sph.normal), dev(sph.weight), dev(q))
    u64 = host(S.dl_eval(*args, trg_xyz=dev(trg), trg_self=dev(tself, torch.int64),
                         subtract=subtract))
    u32 = host(S.dl_eval(*args, trg_xyz=dev(trg), trg_self=dev(tself, torch.int64),
                         subtract=subtract, mixed=True, near_r=near_r))
    assert rel_l2(u64, ref) <= FP64_TOL
    assert rel_max(u32, ref) <= MIXED_TOL


@pytest.mark.parametrize("nt,nphi,R", [(128, 192, 5.0), (128, 192, 12.0)])
def test_dl_mixed_refined_sphere_on_surface(S, oracle_mod, nt, nphi, R):
    """Mixed double layer at the default near radius on a refined sphere with a random
    density, subtracted, at its own points: 24,576 points (the C4 periphery's grid at
    radius 12, and at radius 5 where the grid is finer relative to the curvature).  The
    principal value's cancellation leaves |u| ~ 0.05 |q|; FP32 d.n without the tangent
    band gave 1e-5 here."""
    sph = W.sphere_surface(nt, nphi, R)
    q = np.random.default_rng(int(R) + 70).standard_normal((3, sph.n))
    idx = W.subsample(int(R) + 80, sph.n, 2048)
    ref = oracle_mod.dl(sph.xyz, sph.normal, sph.weight, q, trg_xyz=sph.xyz[:, idx], trg_self=idx,
                        subtract=True, nthreads=NTHREADS)
    args = (dev(sph.xyz), dev(sph.normal), dev(sph.weight), dev(q))
    u64 = host(S.dl_eval(*args))
    u32, d32 = S.dl_eval(*args, mixed=True, diag=True)
    u32 = host(u32)
    e = rel_max(u32[:, idx], ref)
    print(f"sphere {sph.n} R={R}: mixed DL vs oracle {e:.3e}, vs fp64 (all) {rel_max(u32, u64):.3e},"
          f" near pairs {d32.near_pairs}")
    assert rel_l2(u64[:, idx], ref) <= FP64_TOL
    assert e <= MIXED_TOL
    assert rel_max(u32, u64) <= MIXED_TOL


def test_accumulate_and_empty(S, oracle_mod):
    g = _random_fibers(5, 100)
    base = np.random.default_rng(1).standard_normal((3, 100))
    out = dev(base)
    S.sl_eval(dev(g["xyz"]), dev(g["f"]), eps=0.02, accumulate=True, out=out, excl="self")
    ref = oracle_mod.sl(g["xyz"], g["f"], eps=0.02, excl=1)
    assert rel_l2(host(out) - base, ref) <= 1e-12
    # no sources: zeros
    z = host(S.sl_eval(dev(np.zeros((3, 0))), dev(np.zeros((3, 0))), trg_xyz=dev(g["xyz"]),
                       excl=None))
    assert np.all(z == 0)
    # no targets
    e = S.sl_eval(dev(g["xyz"]), dev(g["f"]), trg_xyz=dev(np.zeros((3, 0))), excl=None)
    assert e.shape == (3, 0)


@pytest.mark.parametrize("mixed", [False, True])
def test_dl_ragged_single_and_empty(S, oracle_mod, mixed):
    """The double layer on a ragged surface (91 points: two full tiles and one of 27),
    on a single source, with no sources (zeros, and accumulate leaves the output as it
    was) and with no targets, against the oracle."""
    rng = np.random.default_rng(29)
    tol = FP64_TOL if not mixed else MIXED_TOL
    err = rel_l2 if not mixed else rel_max
    sph = W.sphere_surface(7, 13, 1.1)
    assert sph.n == 91
    q = rng.standard_normal((3, sph.n))
    trg = np.concatenate([sph.xyz, W.uniform_ball(rng, 45, 1.6).T], axis=1)
    tself = np.concatenate([np.arange(sph.n), -np.ones(45, dtype=np.int64)])
    args = (dev(sph.xyz), dev(sph.normal), dev(sph.weight), dev(q))
    for sub in (True, False):
        ref = oracle_mod.dl(sph.xyz, sph.normal, sph.weight, q, trg_xyz=trg, trg_self=tself, subtract=sub)
        u = host(S.dl_eval(*args, trg_xyz=dev(trg), trg_self=dev(tself, torch.int64), subtract=sub,
                           mixed=mixed))
        assert err(u, ref) <= tol
    # one source, off-surface targets
    one = (sph.xyz[:, :1], sph.normal[:, :1], sph.weight[:1], q[:, :1])
    x = W.uniform_ball(rng, 40, 1.6).T
    ref = oracle_mod.dl(*one, trg_xyz=x)
    u = host(S.dl_eval(*(dev(a) for a in one), trg_xyz=dev(x), mixed=mixed))
    assert err(u, ref) <= tol
    # no sources: zeros, and accumulate leaves the output unchanged
    none = (np.zeros((3, 0)), np.zeros((3, 0)), np.zeros(0), np.zeros((3, 0)))
    z = host(S.dl_eval(*(dev(a) for a in none), trg_xyz=dev(x), mixed=mixed))
    assert z.shape == (3, 40) and np.all(z == 0)
    base = rng.standard_normal((3, 40))
    out = dev(base)
    S.dl_eval(*(dev(a) for a in none), trg_xyz=dev(x), mixed=mixed, accumulate=True, out=out)
    assert np.array_equal(host(out), base)
    # no targets
    e = S.dl_eval(*args, trg_xyz=dev(np.zeros((3, 0))), mixed=mixed)
    assert e.shape == (3, 0)


def test_check_inputs_nonfinite_leaves_output_untouched(S):
    g = _random_fibers(6, 64)
    f = g["f"].copy()
    f[1, 5] = np.nan
    out = dev(np.full((3, 64), 7.0))
    with pytest.raises(S.StokesError) as ei:
        S.sl_eval(dev(g["xyz"]), dev(f), eps=0.02, out=out, check_inputs=True)
    assert ei.value.code == S.E_NONFINITE
    assert np.all(host(out) == 7.0)
    fib = g["fib"].copy()
    fib[10] = 0   # decreasing ids
    with pytest.raises(S.StokesError) as ei:
        S.sl_eval(dev(g["xyz"]), dev(g["f"]), src_fiber=dev(fib, torch.int32),
                  fiber_len=dev(g["L"]), eps=0.02, out=out, check_inputs=True)
    assert ei.value.code == S.E_INVAL


def test_coincident_points_skipped_and_counted(S, oracle_mod):
    x = np.array([[0.0, 0.0, 1.0, 0.5], [0.0, 0.0, 0.0, 0.5], [0.0, 0.0, 0.0, 0.5]])
    f = np.random.default_rng(2).standard_normal((3, 4))
    ref, sk = oracle_mod.sl(x, f, excl=1, return_skipped=True)
    for mixed in (False, True):
        u, d = S.sl_eval(dev(x), dev(f), excl="self", mixed=mixed, diag=True)
        u = host(u)
        assert np.all(np.isfinite(u))
        assert d.coincident == sk == 2
        assert d.pairs == 4 * 3 - 2
        assert rel_max(u, ref) <= (1e-14 if not mixed else MIXED_TOL)


def test_local_sbt_gpu(S, oracle_mod):
    rng = np.random.default_rng(4)
    t = W.uniform_sphere_dirs(rng, 1000).T.copy()
    f = rng.standard_normal((3, 1000))
    m = host(S.local_sbt(dev(t), dev(f), 0.01, 0.9))
    mi = host(S.local_sbt(dev(t), dev(f), 0.01, 0.9, inverse=True))
    np.testing.assert_allclose(m, oracle_mod.local_sbt(f, t, 0.01, 0.9), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(mi, oracle_mod.local_sbt_inv(f, t, 0.01, 0.9), rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------------------
# Benchmark-size parity on sampled targets (oracle computes them one by one).
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_config2_sampled(S, oracle_mod):
    c = W.config2()
    fs = c["fibers"]
    a = dict(src_fiber=dev(fs.fiber, torch.int32), fiber_len=dev(fs.length), eps=fs.eps)
    u64 = host(S.sl_eval(dev(fs.xyz), dev(c["force"]), **a))
    u32 = host(S.sl_eval(dev(fs.xyz), dev(c["force"]), mixed=True, **a))   # bench radius
    e_all = rel_max(u32, u64)
    idx = W.subsample(2, fs.n, 4096)
    ref = oracle_mod.sl(fs.xyz, c["force"], src_fiber=fs.fiber, fiber_len=fs.length, eps=fs.eps,
                        trg_xyz=fs.xyz[:, idx], trg_self=idx, excl=1, nthreads=NTHREADS)
    print(f"config2: mixed vs fp64 (all) {e_all:.3e}; fp64 vs oracle {rel_l2(u64[:, idx], ref):.3e};"
          f" mixed vs oracle {rel_max(u32[:, idx], ref):.3e}")
    assert rel_l2(u64[:, idx], ref) <= FP64_TOL
    assert rel_max(u32[:, idx], ref) <= MIXED_TOL
    assert e_all <= MIXED_TOL


@pytest.mark.slow
def test_config4_sampled(S, oracle_mod):
    """Each sum on its own, at the radii the benchmark times (near_r 0): mixed against the
    FP64 GPU path on all 548,864 targets, both against the oracle on 4,096 seeded ones."""
    c = W.config4()
    fs, sph = c["fibers"], c["sphere"]
    trg, sl_self, dl_self = _cfg1_targets(c)
    idx = W.subsample(4, trg.shape[1], 4096)
    res = {}
    for mixed in (False, True):
        u_sl = S.sl_eval(dev(fs.xyz), dev(c["force"]), src_fiber=dev(fs.fiber, torch.int32),
                         fiber_len=dev(fs.length), eps=fs.eps, trg_xyz=dev(trg),
                         trg_self=dev(sl_self, torch.int64), mixed=mixed)
        u_dl = S.dl_eval(dev(sph.xyz), dev(sph.normal), dev(sph.weight), dev(c["q"]), trg_xyz=dev(trg),
                         trg_self=dev(dl_self, torch.int64), mixed=mixed)
        res[mixed] = (host(u_sl), host(u_dl))
    ref_sl = oracle_mod.sl(fs.xyz, c["force"], src_fiber=fs.fiber, fiber_len=fs.length, eps=fs.eps,
                           trg_xyz=trg[:, idx], trg_self=sl_self[idx], excl=1, nthreads=NTHREADS)
    ref_dl = oracle_mod.dl(sph.xyz, sph.normal, sph.weight, c["q"], trg_xyz=trg[:, idx],
                           trg_self=dl_self[idx], subtract=True, nthreads=NTHREADS)
    for k, (name, ref) in enumerate((("SL", ref_sl), ("DL", ref_dl))):
        e_all = rel_max(res[True][k], res[False][k])
        e64 = rel_l2(res[False][k][:, idx], ref)
        e32 = rel_max(res[True][k][:, idx], ref)
        print(f"config4 {name}: mixed vs fp64 (all) {e_all:.3e}; fp64 vs oracle {e64:.3e}; "
              f"mixed vs oracle {e32:.3e}")
        assert e64 <= FP64_TOL
        assert e32 <= MIXED_TOL
        assert e_all <= MIXED_TOL
    # the sphere's own points alone (the principal value of a random density)
    n_f = fs.n
    on = idx[idx >= n_f]
    e_on = rel_max(res[True][1][:, on], ref_dl[:, idx >= n_f])
    print(f"config4 DL at {on.size} sampled sphere points: mixed vs oracle {e_on:.3e}")
    assert e_on <= MIXED_TOL
