"""Exact symmetries of the sums on the GPU path, checked within rounding (the oracle's
own symmetry pins are in test_oracle_pins.py): linearity in the forces and the density,
translation invariance, rotation covariance, source-permutation invariance."""
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


def geom_tol(src, trg, self_idx=None):
    """Bound for a transformed geometry in FP64: moving or rotating the points rounds
    each coordinate again (about eps * max|x| absolute), which perturbs a pair
    difference r by that much, i.e. relatively by eps * max|x| / |r|; the kernels'
    relative sensitivity to r is at most 3 (the doublet's and the stresslet's
    |r|^-3 and |r|^-2 after the r factors), so 8 eps max|x| / min|r| bounds each
    pair's relative change, and the sum's."""
    d = np.sqrt(((trg[:, :, None] - src[:, None, :]) ** 2).sum(0))
    if self_idx is not None:
        i = np.nonzero(self_idx >= 0)[0]
        d[i, self_idx[i]] = np.inf
    R = max(np.abs(src).max(), np.abs(trg).max())
    return 8 * np.finfo(float).eps * R / d.min()


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


@pytest.fixture(scope="module")
def fibers():
    c = W.config0()
    fs = c["fibers"]
    rng = np.random.default_rng(21)
    return fs, c["force"], rng.standard_normal((3, fs.n))


@pytest.fixture(scope="module")
def surface():
    sph = W.sphere_surface(24, 48, 1.3)
    rng = np.random.default_rng(22)
    trg = np.concatenate([sph.xyz, W.uniform_ball(rng, 300, 2.5).T], axis=1)
    tself = np.concatenate([np.arange(sph.n), -np.ones(300, dtype=np.int64)])
    return sph, rng.standard_normal((3, sph.n)), rng.standard_normal((3, sph.n)), trg, tself


def _sl(S, fs, f, xyz=None, mixed=False):
    x = fs.xyz if xyz is None else xyz
    return S.sl_eval(dev(x), dev(f), src_fiber=dev(fs.fiber, torch.int32), fiber_len=dev(fs.length),
                     eps=fs.eps, mixed=mixed).cpu().numpy()


def _dl(S, sph, q, trg, tself, xyz=None, nrm=None, mixed=False):
    y = sph.xyz if xyz is None else xyz
    n = sph.normal if nrm is None else nrm
    return S.dl_eval(dev(y), dev(n), dev(sph.weight), dev(q), trg_xyz=dev(trg),
                     trg_self=dev(tself, torch.int64), mixed=mixed).cpu().numpy()


@pytest.mark.parametrize("mixed,tol", [(False, 1e-13), (True, 4e-6)])
def test_single_layer_linear_translation_rotation(S, fibers, mixed, tol):
    fs, f, g = fibers
    a, b = 0.7, -1.9
    u_f, u_g = _sl(S, fs, f, mixed=mixed), _sl(S, fs, g, mixed=mixed)
    assert rel(_sl(S, fs, a * f + b * g, mixed=mixed), a * u_f + b * u_g) <= tol
    shift = np.array([[3.0], [-1.5], [0.25]])
    t = max(tol, geom_tol(fs.xyz + shift, fs.xyz + shift, np.arange(fs.n)))
    assert rel(_sl(S, fs, f, xyz=fs.xyz + shift, mixed=mixed), u_f) <= t
    Q = _rotation(5)
    t = max(tol, geom_tol(fs.xyz, fs.xyz, np.arange(fs.n)))
    assert rel(_sl(S, fs, Q @ f, xyz=Q @ fs.xyz, mixed=mixed), Q @ u_f) <= t


@pytest.mark.parametrize("mixed,tol", [(False, 1e-13), (True, 4e-6)])
def test_double_layer_linear_translation_rotation(S, surface, mixed, tol):
    sph, q, p, trg, tself = surface
    a, b = -0.4, 2.2
    u_q, u_p = _dl(S, sph, q, trg, tself, mixed=mixed), _dl(S, sph, p, trg, tself, mixed=mixed)
    assert rel(_dl(S, sph, a * q + b * p, trg, tself, mixed=mixed), a * u_q + b * u_p) <= tol
    shift = np.array([[-2.0], [0.5], [1.0]])
    t = max(tol, geom_tol(sph.xyz + shift, trg + shift, tself))
    assert rel(_dl(S, sph, q, trg + shift, tself, xyz=sph.xyz + shift, mixed=mixed), u_q) <= t
    Q = _rotation(6)
    u_rot = _dl(S, sph, Q @ q, Q @ trg, tself, xyz=Q @ sph.xyz, nrm=Q @ sph.normal, mixed=mixed)
    t = max(tol, geom_tol(sph.xyz, trg, tself))
    assert rel(u_rot, Q @ u_q) <= t


def test_source_permutation_invariance(S, fibers, surface):
    """Reordering sources (whole fibers, so that the fiber ids stay contiguous) changes
    only the summation order."""
    fs, f, _ = fibers
    perm_f = np.random.default_rng(7).permutation(fs.n_fib)
    idx = (perm_f[:, None] * fs.nodes_per_fiber + np.arange(fs.nodes_per_fiber)[None, :]).ravel()
    fib_new = np.repeat(np.arange(fs.n_fib, dtype=np.int32), fs.nodes_per_fiber)
    u = S.sl_eval(dev(fs.xyz), dev(f), src_fiber=dev(fs.fiber, torch.int32), fiber_len=dev(fs.length),
                  eps=fs.eps, trg_xyz=dev(fs.xyz), trg_self=dev(np.arange(fs.n), torch.int64)).cpu().numpy()
    inv = np.empty_like(idx)
    inv[idx] = np.arange(fs.n)
    up = S.sl_eval(dev(fs.xyz[:, idx]), dev(f[:, idx]), src_fiber=dev(fib_new, torch.int32),
                   fiber_len=dev(fs.length[perm_f]), eps=fs.eps, trg_xyz=dev(fs.xyz),
                   trg_self=dev(inv.astype(np.int64), torch.int64)).cpu().numpy()
    assert rel(up, u) <= 1e-13
    sph, q, _, trg, tself = surface
    pm = np.random.default_rng(8).permutation(sph.n)
    pinv = np.empty_like(pm)
    pinv[pm] = np.arange(sph.n)
    u = _dl(S, sph, q, trg, tself)
    tself_p = np.where(tself >= 0, pinv[np.maximum(tself, 0)], -1)
    up = S.dl_eval(dev(sph.xyz[:, pm]), dev(sph.normal[:, pm]), dev(sph.weight[pm]), dev(q[:, pm]),
                   trg_xyz=dev(trg), trg_self=dev(tself_p.astype(np.int64), torch.int64)).cpu().numpy()
    assert rel(up, u) <= 1e-13


@pytest.mark.parametrize("mixed,tol", [(False, 1e-12), (True, 4e-6)])
def test_single_layer_reciprocity_at_scale(S, mixed, tol):
    """Reciprocity of the discrete operator (G and W symmetric and even in d; one fiber
    length, so one doublet coefficient) on the confined workload's 32,768 fiber points,
    self-pairs excluded: <g, A f> = <A g, f>.  Each sum's max-norm error e|A f|_inf
    bounds the difference by e (|g|_1 |A f|_inf + |f|_1 |A g|_inf)."""
    c = W.config1()
    fs = c["fibers"]
    assert np.all(fs.length == fs.length[0])
    rng = np.random.default_rng(41)
    f = rng.standard_normal((3, fs.n))
    g = rng.standard_normal((3, fs.n))
    Af, Ag = _sl(S, fs, f, mixed=mixed), _sl(S, fs, g, mixed=mixed)
    lhs, rhs = np.sum(g * Af), np.sum(Ag * f)
    bound = np.abs(g).sum() * np.abs(Af).max() + np.abs(f).sum() * np.abs(Ag).max()
    assert abs(lhs - rhs) <= tol * bound


def _divergence(field, x, h):
    """Central-difference divergence at the columns of x, and its scale (the sum of the
    |du_c/dx_c|), from one evaluation at the six shifted copies of x."""
    n = x.shape[1]
    pts = []
    for c in range(3):
        e = np.zeros((3, 1))
        e[c] = h
        pts += [x + e, x - e]
    u = field(np.concatenate(pts, axis=1))
    div, scale = np.zeros(n), np.zeros(n)
    for c in range(3):
        d = (u[c, (2 * c) * n:(2 * c + 1) * n] - u[c, (2 * c + 1) * n:(2 * c + 2) * n]) / (2 * h)
        div += d
        scale += np.abs(d)
    return div, scale


def test_divergence_free_at_scale(S):
    """The single layer of the confined workload's 32,768 fiber points (all within
    radius 4.92) and the double layer of its 6,144-point sphere (radius 5) are
    divergence free away from their sources: at 96 points on spheres of radius 7 and 2.5
    (FP64; central differences with h = 1e-3 are O((h / distance)^2), below 1e-6 here,
    while a wrong sign or factor in either term leaves a divergence of the scale's order)."""
    c = W.config1()
    fs, sph = c["fibers"], c["sphere"]
    rng = np.random.default_rng(43)
    f = rng.standard_normal((3, fs.n))
    q = rng.standard_normal((3, sph.n))

    def on_sphere(n, r):
        v = rng.standard_normal((3, n))
        return r * v / np.linalg.norm(v, axis=0)

    x_out = on_sphere(96, 7.0)
    sl = lambda y: S.sl_eval(dev(fs.xyz), dev(f), src_fiber=dev(fs.fiber, torch.int32),
                             fiber_len=dev(fs.length), eps=fs.eps, trg_xyz=dev(y), excl="none").cpu().numpy()
    div, scale = _divergence(sl, x_out, 1e-3)
    assert np.all(scale > 0) and np.all(np.abs(div) < 1e-5 * scale)
    for r in (2.5, 7.5):
        x = on_sphere(96, r)
        dl = lambda y: S.dl_eval(dev(sph.xyz), dev(sph.normal), dev(sph.weight), dev(q),
                                 trg_xyz=dev(y)).cpu().numpy()
        div, scale = _divergence(dl, x, 1e-3)
        assert np.all(scale > 0) and np.all(np.abs(div) < 1e-5 * scale)
