"""Seeded synthetic geometries for the Stokes kernel sums.

This module only draws and places points: fiber centerlines sampled at
Chebyshev-Gauss-Lobatto nodes, a confining sphere sampled on a
Gauss-Legendre (in cos theta) x trapezoid (in phi) grid, and i.i.d. normal
forces and densities.  It contains none of the kernel arithmetic, so both the
GPU library and the CPU oracle can take their inputs from here.

Conventions (paper, section "Fiber representation", eq. cheb-basis):
  * a fiber with p+1 nodes uses alpha_k = cos(k pi / p), k = 0..p; node k sits
    at s = (alpha_k + 1) L / 2 along the fiber, so k = 0 is the plus end s = L.
  * straight fibers: X_k = X(s=0) + s_k t, with unit tangent t = X_s.

All arrays are structure-of-arrays float64: positions are (3, N).
Random streams: ``numpy.random.Generator(PCG64)`` children of
``SeedSequence(seed)``: child 0 draws geometry (including rejection resampling),
child 1 draws forces / densities, child 2 draws anything else (subsamples).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "FiberSet", "SphereSurface", "cgl_alpha", "uniform_ball", "uniform_sphere_dirs",
    "straight_fibers", "sphere_surface", "config0", "config1", "config2", "config4",
    "serving_request", "serving_stream", "random_points", "bent_fibers", "config_step",
]


def _streams(seed, n=3):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def cgl_alpha(p: int) -> np.ndarray:
    """Chebyshev-Gauss-Lobatto collocation points alpha_k = cos(k pi/p), k=0..p."""
    k = np.arange(p + 1, dtype=np.float64)
    return np.cos(k * np.pi / p)


def uniform_sphere_dirs(rng, n: int) -> np.ndarray:
    """n unit vectors uniform on S^2, shape (n, 3)."""
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def uniform_ball(rng, n: int, R: float, r_min: float = 0.0) -> np.ndarray:
    """n points uniform (in volume) in the shell r_min <= r <= R, shape (n, 3)."""
    d = uniform_sphere_dirs(rng, n)
    u = rng.random(n)
    r = (r_min ** 3 + u * (R ** 3 - r_min ** 3)) ** (1.0 / 3.0)
    return d * r[:, None]


def cone_dirs(rng, n: int, axis, half_angle: float) -> np.ndarray:
    """n unit vectors uniform on the spherical cap of the given half angle about axis."""
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    cz = rng.uniform(math.cos(half_angle), 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    # orthonormal frame (e1, e2, axis)
    helper = np.array([0.0, 0.0, 1.0]) if abs(axis[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(axis, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(axis, e1)
    return (cz[:, None] * axis[None, :] + (sz * np.cos(phi))[:, None] * e1[None, :]
            + (sz * np.sin(phi))[:, None] * e2[None, :])


@dataclasses.dataclass
class FiberSet:
    """Straight fibers sampled at CGL nodes, fiber-contiguous ordering."""
    xyz: np.ndarray          # (3, N) node positions
    tangent: np.ndarray      # (3, N) unit tangent X_s at each node
    fiber: np.ndarray        # (N,) int32 fiber id, non-decreasing
    length: np.ndarray       # (n_fib,) fiber lengths L_m
    nodes_per_fiber: int
    eps: float

    @property
    def n(self) -> int:
        return self.xyz.shape[1]

    @property
    def n_fib(self) -> int:
        return self.length.shape[0]


@dataclasses.dataclass
class SphereSurface:
    """Quadrature points of a sphere of radius R centred at the origin."""
    xyz: np.ndarray          # (3, M)
    normal: np.ndarray       # (3, M) outward unit normal
    weight: np.ndarray       # (M,) area weights
    R: float

    @property
    def n(self) -> int:
        return self.xyz.shape[1]


def straight_fibers(minus_end: np.ndarray, tangent: np.ndarray, length: np.ndarray,
                    nodes_per_fiber: int) -> np.ndarray:
    """Node positions (n_fib, nodes, 3) of straight fibers from their minus ends."""
    p = nodes_per_fiber - 1
    alpha = cgl_alpha(p)
    s = (alpha[None, :] + 1.0) * 0.5 * length[:, None]          # (n_fib, nodes)
    return minus_end[:, None, :] + s[:, :, None] * tangent[:, None, :]


def _fiber_nodes_centered(center, tangent, length, nodes):
    minus = center - 0.5 * length[:, None] * tangent
    return straight_fibers(minus, tangent, length, nodes)


def _resolve_overlaps(nodes_fn, params, resample_fn, gap, max_rounds=200):
    """Resample fibers until no two nodes of different fibers are closer than gap.

    nodes_fn(params) -> (n_fib, nodes, 3); resample_fn(params, idx) redraws the
    fibers listed in idx in place (in increasing index order).  For every
    conflicting pair the fiber with the larger index is redrawn, so the fiber
    with the smaller index is kept and the result is deterministic.
    """
    from scipy.spatial import cKDTree
    for _ in range(max_rounds):
        nodes = nodes_fn(params)
        n_fib, npf, _ = nodes.shape
        pts = nodes.reshape(-1, 3)
        pairs = cKDTree(pts).query_pairs(gap, output_type="ndarray")
        if pairs.size:
            fa = pairs[:, 0] // npf
            fb = pairs[:, 1] // npf
            other = fa != fb
            bad = np.unique(np.maximum(fa[other], fb[other]))
        else:
            bad = np.zeros(0, dtype=np.int64)
        if bad.size == 0:
            return nodes
        resample_fn(params, bad)
    raise RuntimeError("fiber placement did not converge")


def _fiberset(nodes, tangent, length, eps):
    n_fib, npf, _ = nodes.shape
    xyz = np.ascontiguousarray(nodes.reshape(-1, 3).T)
    tan = np.ascontiguousarray(np.repeat(tangent, npf, axis=0).T)
    fib = np.repeat(np.arange(n_fib, dtype=np.int32), npf)
    return FiberSet(xyz=xyz, tangent=tan, fiber=fib, length=np.asarray(length, np.float64).copy(),
                    nodes_per_fiber=npf, eps=eps)


def random_fibers_in_ball(rng, n_fib, nodes, R_center, L=1.0, eps=0.01, gap=None,
                          shell_fraction=0.0, shell_inner=None):
    """Fibers of length L with centres uniform in a ball (optionally a shell share).

    shell_fraction of the fibers (the last ones) get centres uniform in the
    shell shell_inner <= r <= R_center.  gap: minimum node distance between
    different fibers (None = no rejection).
    """
    n_shell = int(round(shell_fraction * n_fib))
    n_core = n_fib - n_shell
    length = np.full(n_fib, float(L))

    def draw_centers(idx):
        c = np.empty((len(idx), 3))
        core = idx < n_core
        if core.any():
            c[core] = uniform_ball(rng, int(core.sum()), R_center)
        if (~core).any():
            c[~core] = uniform_ball(rng, int((~core).sum()), R_center, r_min=shell_inner)
        return c

    allidx = np.arange(n_fib)
    params = {"c": draw_centers(allidx), "t": uniform_sphere_dirs(rng, n_fib)}

    def nodes_fn(p):
        return _fiber_nodes_centered(p["c"], p["t"], length, nodes)

    def resample(p, idx):
        p["c"][idx] = draw_centers(idx)
        p["t"][idx] = uniform_sphere_dirs(rng, len(idx))

    if gap is None:
        pts = nodes_fn(params)
    else:
        pts = _resolve_overlaps(nodes_fn, params, resample, gap)
    return _fiberset(pts, params["t"], length, eps)


def bent_shape(nodes, L, amp):
    """Planar centerlines of length L parametrised by arclength, (len(amp), nodes, 2) in
    their own frames, each centred on its mean node: tangent angle
    theta(s) = amp (phi(s/L) - 1/2) with phi(u) = u^3 (10 - 15 u + 6 u^2), so
    theta' = theta'' = 0 at both ends (zero curvature and curvature derivative:
    compatible with free ends).  Positions are the integrals of (cos theta, sin theta),
    by 48-point Gauss-Legendre on [0, s_k]."""
    amp = np.atleast_1d(np.asarray(amp, np.float64))
    s = (cgl_alpha(nodes - 1) + 1.0) * 0.5 * L
    gx, gw = np.polynomial.legendre.leggauss(48)
    q = 0.5 * s[:, None] * (gx[None, :] + 1.0)               # (nodes, 48) points in [0, s_k]
    u = q / L
    th = amp[:, None, None] * (u ** 3 * (10.0 - 15.0 * u + 6.0 * u * u) - 0.5)[None]
    w = (0.5 * s[:, None] * gw[None, :])[None]
    xy = np.stack([np.sum(w * np.cos(th), axis=2), np.sum(w * np.sin(th), axis=2)], axis=2)
    return xy - xy.mean(axis=1, keepdims=True)


def bent_fibers(rng, n_fib, nodes, R_center, L=1.0, eps=0.01, amp=0.6, gap=None):
    """Bent planar fibers (bent_shape with amp uniform in [-amp, amp]) with centres
    uniform in a ball, random orientation of the shape's plane and axis.  gap: minimum
    node distance between different fibers (None = no rejection).  The FiberSet's
    tangent is the chord direction (the time step computes its own tangents)."""
    length = np.full(n_fib, float(L))

    def draw(idx):
        k = len(idx)
        t = uniform_sphere_dirs(rng, k)
        a = uniform_sphere_dirs(rng, k)
        nrm = np.cross(t, a)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        return uniform_ball(rng, k, R_center), t, nrm, rng.uniform(-amp, amp, k)

    params = dict(zip(("c", "t", "n", "amp"), draw(np.arange(n_fib))))

    def nodes_fn(p):
        xy = bent_shape(nodes, L, p["amp"])
        return (p["c"][:, None, :] + xy[:, :, :1] * p["t"][:, None, :]
                + xy[:, :, 1:] * p["n"][:, None, :])

    def resample(p, idx):
        c, t, nrm, am = draw(idx)
        p["c"][idx], p["t"][idx], p["n"][idx], p["amp"][idx] = c, t, nrm, am

    pts = nodes_fn(params) if gap is None else _resolve_overlaps(nodes_fn, params, resample, gap)
    return _fiberset(pts, params["t"], length, eps)


def config_step(seed=5, n_fib=2048, nodes=32, R=5.0, L=1.0, eps=0.01, E=1.0, mu=1.0):
    """One implicit step of a sedimenting suspension of free bent fibers: n_fib fibers
    x nodes CGL nodes (the paper's GMRES study uses up to 2048 fibers of 31 points),
    centres in a ball of radius R (gap 0.05 between fibers), uniform force density
    -E/(32 L^3) e_z plus a seeded random part of the same size, and the step
    dt = 1e-3 tau_E with tau_E = -8 pi mu L^4 / (E ln(eps^2 e)) (section "Numerical
    results": stable steps of 0.25e-3 .. 1.3e-3 tau_E)."""
    g, d, _ = _streams(seed)
    fs = bent_fibers(g, n_fib, nodes, R - 0.55 * L, L=L, eps=eps, gap=0.05 * L)
    f0 = E / (32.0 * L ** 3)
    f_ext = f0 * (d.standard_normal((3, fs.n)) * 0.5 + np.array([[0.0], [0.0], [-1.0]]))
    tau = -8.0 * math.pi * mu * L ** 4 / (E * math.log(eps * eps * math.e))
    return {"fibers": fs, "f_ext": f_ext, "E": E, "mu": mu, "eps": eps, "dt": 1e-3 * tau}


def sphere_surface(n_theta: int, n_phi: int, R: float, patch=(4, 8)) -> SphereSurface:
    """Gauss-Legendre (in cos theta) x trapezoid (in phi) points on a sphere.

    Points are ordered in patches of patch[0] theta x patch[1] phi nodes
    (patch-major, then theta, then phi), so consecutive runs of
    patch[0]*patch[1] points are spatially compact.  Weights are
    R^2 w_GL 2 pi / n_phi; normals point outward (y / R).
    """
    x, w = np.polynomial.legendre.leggauss(n_theta)          # x = cos(theta)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    pt, pp = patch
    if n_theta % pt or n_phi % pp:
        pt, pp = 1, n_phi
    order = []
    for I in range(n_theta // pt):
        for J in range(n_phi // pp):
            for i in range(I * pt, (I + 1) * pt):
                for j in range(J * pp, (J + 1) * pp):
                    order.append((i, j))
    ii = np.array([o[0] for o in order])
    jj = np.array([o[1] for o in order])
    ct = x[ii]
    st = np.sqrt(1.0 - ct * ct)
    nrm = np.stack([st * np.cos(phi[jj]), st * np.sin(phi[jj]), ct])
    wt = R * R * w[ii] * (2.0 * np.pi / n_phi)
    return SphereSurface(xyz=R * nrm, normal=nrm.copy(), weight=wt, R=float(R))


def random_points(seed, n, R=1.0):
    """n points uniform in a ball, (3, n); forces N(0,1) (3, n)."""
    g, d, _ = _streams(seed)
    return np.ascontiguousarray(uniform_ball(g, n, R).T), d.standard_normal((3, n))


# ---------------------------------------------------------------------------
# Named workloads (seeded).  Sizes follow the benchmark configurations.
# ---------------------------------------------------------------------------

def config0(seed=0):
    """16 fibers x 32 CGL nodes, L=1, eps=0.01, centres uniform in a ball of radius 3."""
    g, d, _ = _streams(seed)
    fs = random_fibers_in_ball(g, 16, 32, 3.0, L=1.0, eps=0.01)
    force = d.standard_normal((3, fs.n))
    return {"fibers": fs, "force": force, "mu": 1.0, "eps": 0.01}


def config1(seed=1, n_fib=1024, n_theta=64, n_phi=96, R=5.0):
    """Confined: fibers in a sphere of radius R (gap 0.05 to wall and between fibers)."""
    g, d, _ = _streams(seed)
    fs = random_fibers_in_ball(g, n_fib, 32, R - 0.55, L=1.0, eps=0.01, gap=0.05)
    sph = sphere_surface(n_theta, n_phi, R)
    force = d.standard_normal((3, fs.n))
    q = d.standard_normal((3, sph.n))
    return {"fibers": fs, "force": force, "sphere": sph, "q": q, "mu": 1.0, "eps": 0.01}


def config2(seed=2, fibers_per_pole=2048, nodes=64, half_angle_deg=30.0, gap=0.005):
    """Spindle: fibers radiating from poles (+-4,0,0) toward the other pole."""
    g, d, _ = _streams(seed)
    n_fib = 2 * fibers_per_pole
    pole = np.zeros((n_fib, 3))
    pole[:fibers_per_pole, 0] = 4.0
    pole[fibers_per_pole:, 0] = -4.0
    axis_sign = np.where(np.arange(n_fib) < fibers_per_pole, -1.0, 1.0)
    ha = math.radians(half_angle_deg)

    def draw(idx):
        t = np.empty((len(idx), 3))
        for sgn in (-1.0, 1.0):
            m = axis_sign[idx] == sgn
            if m.any():
                t[m] = cone_dirs(g, int(m.sum()), [sgn, 0.0, 0.0], ha)
        L = g.uniform(1.0, 6.0, len(idx))
        return t, L

    t0, L0 = draw(np.arange(n_fib))
    params = {"t": t0, "L": L0}

    def nodes_fn(p):
        minus = pole + 0.5 * p["t"]
        return straight_fibers(minus, p["t"], p["L"], nodes)

    def resample(p, idx):
        t, L = draw(idx)
        p["t"][idx] = t
        p["L"][idx] = L

    pts = _resolve_overlaps(nodes_fn, params, resample, gap)
    fs = _fiberset(pts, params["t"], params["L"], 0.005)
    force = d.standard_normal((3, fs.n)) / fs.length[fs.fiber][None, :]
    return {"fibers": fs, "force": force, "mu": 1.0, "eps": 0.005}


def config4(seed=4, n_fib=16384, n_theta=128, n_phi=192, R=12.0, shell_fraction=0.3):
    """Large confined: 30% of the fibers centred within 1.0 of the wall."""
    g, d, x = _streams(seed)
    fs = random_fibers_in_ball(g, n_fib, 32, R - 0.55, L=1.0, eps=0.01, gap=0.05,
                               shell_fraction=shell_fraction, shell_inner=R - 1.0)
    sph = sphere_surface(n_theta, n_phi, R)
    force = d.standard_normal((3, fs.n))
    q = d.standard_normal((3, sph.n))
    return {"fibers": fs, "force": force, "sphere": sph, "q": q, "mu": 1.0, "eps": 0.01,
            "rng_extra": x}


def subsample(seed, n_total, k):
    """k distinct sorted indices out of n_total (seeded, stream 2)."""
    _, _, x = _streams(seed)
    return np.sort(x.choice(n_total, size=min(k, n_total), replace=False)).astype(np.int64)


def serving_request(seed, rid, n_fib: Optional[int] = None, nodes: Optional[int] = None,
                    iters: Optional[int] = None):
    """One mobility-solve request: random fibers as in config 0, in a ball 2 N_f^(1/3)."""
    g, d, _ = _streams([seed, rid])
    if n_fib is None:
        n_fib = int(round(math.exp(g.uniform(math.log(32), math.log(2048)))))
    if nodes is None:
        nodes = int(g.choice([16, 32, 64]))
    if iters is None:
        iters = int(g.integers(20, 61))
    fs = random_fibers_in_ball(g, n_fib, nodes, 2.0 * n_fib ** (1.0 / 3.0), L=1.0, eps=0.01)
    rhs = d.standard_normal((3, fs.n))
    return {"fibers": fs, "rhs": rhs, "iters": iters, "mu": 1.0, "eps": 0.01, "rid": rid}


def serving_stream(seed, n_req, rate):
    """Poisson arrival times (seconds) for n_req requests at the given rate."""
    _, _, x = _streams([seed, 1 << 30])
    return np.cumsum(x.exponential(1.0 / rate, n_req))
