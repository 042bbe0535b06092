"""Oracle for the Stokes kernel sums, the local slender-body operator and GMRES.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product library never
calls it and shares no code with it; the two only share the seeded input
generators, which hold none of the method's arithmetic.

Contents
  * ``sl`` / ``dl``: the brute-force FP64 double loops of ``stokes_oracle.c``
    (single layer: Stokeslet + doublet, eq. oseen / eq. main-sb-vel; double
    layer: eq. double-layer with the stresslet, and on-surface singularity
    subtraction).
  * ``local_sbt`` / ``local_sbt_inv``: the local slender-body operator M of
    eq. main-sb-local and its inverse (the 3x3 fiber-node blocks of the
    block-Jacobi preconditioner, eq. prec, in their local form).
  * ``clenshaw_curtis``: Clenshaw-Curtis weights on CGL nodes (section
    "Integration over fiber centerlines"), as the interpolatory rule.
  * ``nonlocal_sbt``: the regularised finite-part self-interaction K_delta of
    eq. sb-stokes-reg on each fiber, with the Clenshaw-Curtis rule of section
    "Integration over fiber centerlines" (the s' = s term vanishes: both parts of
    the integrand tend to (I + X_s X_s) f(s) / (8 pi mu delta) there).
  * ``fiber_block_solve``: the fiber block-Jacobi preconditioner of section
    "Linear solver and preconditioner": each fiber's self block M + K_delta is
    formed column by column and solved with numpy.linalg.solve.
  * ``mobility_apply`` / ``gmres``: the fiber mobility operator
    A f = M f [+ K_delta f] + u_bar[f] (eq. main-sb-local, with the complementary
    flow of eq. complementary-uf: all other fibers) and right-preconditioned
    GMRES (Saad) with classical Gram-Schmidt applied twice and Givens rotations.

Nothing here is blocked, fused or reordered beyond the definitions.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Callable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stokes_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")
# A test may point the oracle at a deliberately broken build of the same source
# (mutation test of the pins); the variable is never set otherwise.
_LIB = os.environ.get("STOKES_ORACLE_LIB", _LIB_DEFAULT)
_lib = None

EXCL_NONE, EXCL_SELF_POINT, EXCL_SAME_FIBER = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, FP64, no fast-math, OpenMP)."""
    return compile_c(_SRC, _LIB_DEFAULT, force)


def compile_c(src: str, out: str, force: bool = True) -> str:
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-ffp-contract=off", src, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is None:
        if _LIB == _LIB_DEFAULT and (not os.path.exists(_LIB)
                                     or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_sl.restype = ctypes.c_int64
        lib.oracle_sl.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_int64, P, P, P,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                  P, ctypes.c_int]
        lib.oracle_dl.restype = ctypes.c_int64
        lib.oracle_dl.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int64, P, P, ctypes.c_int,
                                  P, ctypes.c_int]
        lib.oracle_has_openmp.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int64)


def sl(src_xyz, src_force, *, src_weight=None, src_fiber=None, fiber_len=None,
       trg_xyz=None, trg_self=None, trg_fiber=None, mu=1.0, eps=0.01,
       excl=EXCL_SELF_POINT, doublet=True, nthreads=1, return_skipped=False):
    """Stokeslet + doublet single-layer sum at the targets, (3, n_trg) float64."""
    lib = _load()
    sx = _f64(src_xyz)
    ns = sx.shape[1]
    f = _f64(src_force, (3, ns))
    w = _f64(src_weight)
    sfib = _i32(src_fiber)
    flen = _f64(fiber_len)
    tx = _f64(trg_xyz)
    nt = ns if tx is None else tx.shape[1]
    ts = _i64(trg_self)
    tf = _i32(trg_fiber)
    u = np.empty((3, nt), dtype=np.float64)
    skipped = lib.oracle_sl(ns, _ptr(sx), _ptr(f), _ptr(w), _ptr(sfib), _ptr(flen), nt, _ptr(tx),
                            _ptr(ts), _ptr(tf), float(mu), float(eps), int(excl), int(bool(doublet)),
                            _ptr(u), int(nthreads))
    return (u, skipped) if return_skipped else u


def dl(src_xyz, src_normal, src_weight, src_q, *, trg_xyz=None, trg_self=None, subtract=True,
       nthreads=1, return_skipped=False):
    """Stresslet double-layer sum at the targets, (3, n_trg) float64."""
    lib = _load()
    sx = _f64(src_xyz)
    ns = sx.shape[1]
    n = _f64(src_normal, (3, ns))
    w = _f64(src_weight, (ns,))
    q = _f64(src_q, (3, ns))
    tx = _f64(trg_xyz)
    nt = ns if tx is None else tx.shape[1]
    ts = _i64(trg_self)
    u = np.empty((3, nt), dtype=np.float64)
    skipped = lib.oracle_dl(ns, _ptr(sx), _ptr(n), _ptr(w), _ptr(q), nt, _ptr(tx), _ptr(ts),
                            int(bool(subtract)), _ptr(u), int(nthreads))
    return (u, skipped) if return_skipped else u


def has_openmp() -> bool:
    return bool(_load().oracle_has_openmp())


# ---------------------------------------------------------------------------
# Local slender-body operator (eq. main-sb-local) and its inverse.
# ---------------------------------------------------------------------------

def local_sbt(f, tangent, eps, mu=1.0):
    """M f = (1/(8 pi mu)) [ -ln(eps^2 e) (I + t t) + 2 (I - t t) ] f at every node."""
    f = np.asarray(f, dtype=np.float64)
    t = np.asarray(tangent, dtype=np.float64)
    tf = np.sum(t * f, axis=0)
    ttf = t * tf[None, :]
    L = -math.log(eps * eps * math.e)
    return (L * (f + ttf) + 2.0 * (f - ttf)) / (8.0 * math.pi * mu)


def local_sbt_inv(v, tangent, eps, mu=1.0):
    """M^{-1} v, by solving the 3x3 system of every node with numpy.linalg.solve."""
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(tangent, dtype=np.float64)
    L = -math.log(eps * eps * math.e)
    n = v.shape[1]
    out = np.empty_like(v)
    eye = np.eye(3)
    for i in range(n):
        tt = np.outer(t[:, i], t[:, i])
        Mi = (L * (eye + tt) + 2.0 * (eye - tt)) / (8.0 * math.pi * mu)
        out[:, i] = np.linalg.solve(Mi, v[:, i])
    return out


# ---------------------------------------------------------------------------
# Clenshaw-Curtis quadrature on the CGL nodes alpha_k = cos(k pi / p).
# ---------------------------------------------------------------------------

def clenshaw_curtis(p: int) -> np.ndarray:
    """Weights of the interpolatory rule on CGL nodes: exact for every polynomial of
    degree <= p.  Solved from the moment equations sum_k w_k T_m(alpha_k) = int T_m."""
    k = np.arange(p + 1)
    alpha = np.cos(k * np.pi / p)
    m = np.arange(p + 1)
    V = np.cos(np.outer(m, np.arccos(np.clip(alpha, -1.0, 1.0))))     # V[m, k] = T_m(alpha_k)
    mom = np.where(m % 2 == 0, 2.0 / (1.0 - m.astype(np.float64) ** 2 + (m % 2)), 0.0)
    return np.linalg.solve(V, mom)


def fiber_quadrature_weights(fiber, fiber_len, nodes_per_fiber):
    """Per-node weights for int_0^L ds: Clenshaw-Curtis weights times L/2."""
    w = clenshaw_curtis(nodes_per_fiber - 1)
    fiber = np.asarray(fiber)
    kk = np.arange(fiber.shape[0]) % nodes_per_fiber
    return w[kk] * 0.5 * np.asarray(fiber_len, dtype=np.float64)[fiber]


# ---------------------------------------------------------------------------
# Fiber mobility operator and GMRES.
# ---------------------------------------------------------------------------

def fiber_arclength(fiber, fiber_len, nodes_per_fiber):
    """Arc length s of every node: node k of a fiber sits at alpha_k = cos(k pi / p),
    s = (L/2)(1 + alpha_k), so node 0 is the plus end s = L."""
    p = nodes_per_fiber - 1
    fiber = np.asarray(fiber)
    kk = np.arange(fiber.shape[0]) % nodes_per_fiber
    return 0.5 * np.asarray(fiber_len, dtype=np.float64)[fiber] * (1.0 + np.cos(kk * np.pi / p))


def nonlocal_sbt(f, xyz, tangent, fiber, fiber_len, nodes_per_fiber, delta, mu=1.0):
    """K_delta[f] at every node (eq. sb-stokes-reg): over the node's own fiber,

        sum_{k != i} w_k [ |r|/sqrt(|r|^2 + delta^2) G(r) f_k
                           - (I + t_i t_i) f_i / (8 pi mu sqrt((s_i - s_k)^2 + delta^2)) ],

    r = X_i - X_k, G(r) = (I/|r| + r r/|r|^3)/(8 pi mu), w_k the Clenshaw-Curtis
    weight times L/2 and s the arc length.  Plain loops over fibers and node pairs."""
    f = np.asarray(f, dtype=np.float64)
    X = np.asarray(xyz, dtype=np.float64)
    t = np.asarray(tangent, dtype=np.float64)
    fiber = np.asarray(fiber)
    w = fiber_quadrature_weights(fiber, fiber_len, nodes_per_fiber)
    s = fiber_arclength(fiber, fiber_len, nodes_per_fiber)
    c = 1.0 / (8.0 * math.pi * mu)
    out = np.zeros_like(f)
    n_fib = int(fiber.max()) + 1 if fiber.size else 0
    for m in range(n_fib):
        idx = np.nonzero(fiber == m)[0]
        for i in idx:
            ks = idx[idx != i]                                      # the s' = s term is zero
            ti = t[:, i]
            proj_fi = f[:, i] + ti * np.dot(ti, f[:, i])           # (I + t_i t_i) f_i
            r = X[:, i:i + 1] - X[:, ks]                            # (3, n-1)
            rn = np.sqrt(np.sum(r * r, axis=0))
            rf = np.sum(r * f[:, ks], axis=0)
            G_fk = c * (f[:, ks] / rn + r * (rf / rn ** 3))
            phi = rn / np.sqrt(rn * rn + delta * delta)
            psi = 1.0 / np.sqrt((s[i] - s[ks]) ** 2 + delta * delta)
            out[:, i] = np.sum(w[ks] * (phi * G_fk - c * proj_fi[:, None] * psi), axis=1)
    return out


def fiber_blocks(xyz, tangent, fiber, fiber_len, nodes_per_fiber, eps, mu=1.0, delta=None):
    """Self block M [+ K_delta] of every fiber, as (node indices, 3n x 3n matrix) with
    row and column index c n + k (component c of the fiber's node k).  Each column is
    the operator applied to a unit vector of the fiber."""
    fiber = np.asarray(fiber)
    blocks = []
    n_fib = int(fiber.max()) + 1 if fiber.size else 0
    for m in range(n_fib):
        idx = np.nonzero(fiber == m)[0]
        n = idx.size
        X, t = np.asarray(xyz)[:, idx], np.asarray(tangent)[:, idx]
        fl = np.asarray(fiber_len, dtype=np.float64)[m: m + 1]
        fb = np.zeros(n, dtype=np.int64)
        B = np.empty((3 * n, 3 * n))
        for col in range(3 * n):
            e = np.zeros((3, n))
            e.flat[col] = 1.0
            Ae = local_sbt(e, t, eps, mu)
            if delta is not None:
                Ae = Ae + nonlocal_sbt(e, X, t, fb, fl, nodes_per_fiber, delta, mu)
            B[:, col] = Ae.ravel()
        blocks.append((idx, B))
    return blocks


def fiber_block_solve(v, blocks):
    """Block-Jacobi preconditioner: z with B_m z_m = v_m on every fiber m (Gaussian
    elimination, numpy.linalg.solve), blocks from ``fiber_blocks``."""
    v = np.asarray(v, dtype=np.float64)
    out = np.empty_like(v)
    for idx, B in blocks:
        out[:, idx] = np.linalg.solve(B, v[:, idx].ravel()).reshape(3, idx.size)
    return out


def mobility_apply(f, xyz, tangent, fiber, fiber_len, nodes_per_fiber, eps, mu=1.0,
                   doublet=True, nthreads=1, delta=None):
    """A f = M f [+ K_delta f] + u_bar[f]: local SBT term, the nonlocal self term when
    delta is given, and the flow of all other fibers (Clenshaw-Curtis-weighted
    Stokeslet + doublet sum, own fiber excluded)."""
    w = fiber_quadrature_weights(fiber, fiber_len, nodes_per_fiber)
    u = sl(xyz, f, src_weight=w, src_fiber=fiber, fiber_len=fiber_len, mu=mu, eps=eps,
           excl=EXCL_SAME_FIBER, doublet=doublet, nthreads=nthreads)
    out = local_sbt(f, tangent, eps, mu) + u
    if delta is not None:
        out = out + nonlocal_sbt(f, xyz, tangent, fiber, fiber_len, nodes_per_fiber, delta, mu)
    return out


def gmres(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, k: int,
          apply_Pinv: Optional[Callable[[np.ndarray], np.ndarray]] = None):
    """Right-preconditioned GMRES(k) from x0 = 0 (Saad, Alg. 6.9 with Givens rotations).

    Solves A P^{-1} y = b by Arnoldi with classical Gram-Schmidt applied twice,
    and returns x = P^{-1} y.  Stops early only on exact breakdown (h_{j+1,j} = 0).
    Returns (x, residual_history, iterations); residual_history[j] = |g_j|, the
    least-squares residual norm after j iterations.
    """
    b = np.asarray(b, dtype=np.float64).ravel()
    P = apply_Pinv if apply_Pinv is not None else (lambda v: v)
    n = b.size
    beta = float(np.sqrt(np.dot(b, b)))
    if beta == 0.0:
        return np.zeros(n), [0.0], 0
    V = np.zeros((k + 1, n))
    H = np.zeros((k + 1, k))
    cs = np.zeros(k)
    sn = np.zeros(k)
    g = np.zeros(k + 1)
    g[0] = beta
    V[0] = b / beta
    hist = [beta]
    m = 0
    for j in range(k):
        w = apply_A(P(V[j]))
        h = V[: j + 1] @ w
        w = w - V[: j + 1].T @ h
        h2 = V[: j + 1] @ w
        w = w - V[: j + 1].T @ h2
        h = h + h2
        hn = float(np.sqrt(np.dot(w, w)))
        col = np.concatenate([h, [hn]])
        for i in range(j):
            a, c = col[i], col[i + 1]
            col[i] = cs[i] * a + sn[i] * c
            col[i + 1] = -sn[i] * a + cs[i] * c
        den = math.hypot(col[j], col[j + 1])
        cs[j] = col[j] / den
        sn[j] = col[j + 1] / den
        col[j] = den
        col[j + 1] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        H[: j + 2, j] = col
        hist.append(abs(g[j + 1]))
        m = j + 1
        if hn == 0.0:
            break
        V[j + 1] = w / hn
    y = np.zeros(m)
    for i in range(m - 1, -1, -1):             # back substitution R y = g
        y[i] = (g[i] - np.dot(H[i, i + 1: m], y[i + 1: m])) / H[i, i]
    x = P(V[:m].T @ y)
    return x, hist, m


def mobility_solve(rhs, xyz, tangent, fiber, fiber_len, nodes_per_fiber, eps, iters, mu=1.0,
                   doublet=True, nthreads=1, delta=None, precond="local"):
    """GMRES on A f = V with a right preconditioner: "local" applies M^{-1} node by
    node, "block" solves each fiber's self block M [+ K_delta].  delta given: the
    operator includes the nonlocal self term K_delta."""
    shape = np.asarray(rhs).shape

    def A(v):
        return mobility_apply(v.reshape(shape), xyz, tangent, fiber, fiber_len, nodes_per_fiber,
                              eps, mu, doublet, nthreads, delta).ravel()

    if precond == "block":
        blocks = fiber_blocks(xyz, tangent, fiber, fiber_len, nodes_per_fiber, eps, mu, delta)

        def Pinv(v):
            return fiber_block_solve(v.reshape(shape), blocks).ravel()
    elif precond == "local":
        def Pinv(v):
            return local_sbt_inv_closed(v.reshape(shape), tangent, eps, mu).ravel()
    else:
        raise ValueError(f"unknown preconditioner {precond!r}")

    x, hist, m = gmres(A, np.asarray(rhs).ravel(), iters, Pinv)
    return x.reshape(shape), hist, m


def local_sbt_inv_closed(v, tangent, eps, mu=1.0):
    """M^{-1} v from the spectral decomposition of the 3x3 block: eigenvalue
    2 kappa/(8 pi mu) along t and (kappa+2)/(8 pi mu) across, kappa = -ln(eps^2 e).
    (Checked against ``local_sbt_inv`` in the tests.)"""
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(tangent, dtype=np.float64)
    kap = -math.log(eps * eps * math.e)
    tv = np.sum(t * v, axis=0)
    par = t * tv[None, :]
    return 8.0 * math.pi * mu * (par / (2.0 * kap) + (v - par) / (kap + 2.0))


# Confined rigid particles (second-kind boundary integral mobility problem).
from .particles import ParticleSystem, particle_solve, stokeslet, rotlet, dl_diagonal  # noqa: E402,F401

# One implicit time step of free elastic fibers.
from .timestep import FiberStep, cheb_diff, fiber_step  # noqa: E402,F401
