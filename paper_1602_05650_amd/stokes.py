"""ctypes binding of libstokes.so (C ABI in include/stokes.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Device arrays are torch tensors on a ROCm device
(float64 SoA planes of shape (3, n), int32 fiber ids, int64 self indices);
streams are torch.cuda streams.  If the library is missing this module raises
at import: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstokes.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NONFINITE, E_BUSY, E_CANCELED, E_TIMEOUT, E_NOTFOUND = range(9)
PREC_FP64 = 0
PREC_MIXED = 1
EXCL_SELF_POINT = 2
EXCL_SAME_FIBER = 4
NO_DOUBLET = 8
ACCUMULATE = 16
CHECK_INPUTS = 32
ONSURF_RAW = 64
NONLOCAL = 128
PRECOND_BLOCK = 256
EAGER = 512
MAX_ITERS = 128


class StokesError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{status_string(code)}: {msg}")
        self.code = code


class Diag(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("near_pairs", ctypes.c_int64),
                ("coincident", ctypes.c_int64)]


class SessionCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("max_queue", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("device", ctypes.c_int32), ("step_pairs", ctypes.c_int64)]


class SolveReq(ctypes.Structure):
    _fields_ = [("n_fib", ctypes.c_int32), ("nodes_per_fib", ctypes.c_int32),
                ("xyz", ctypes.c_void_p), ("tangent", ctypes.c_void_p),
                ("fiber_len", ctypes.c_void_p), ("rhs", ctypes.c_void_p),
                ("eps", ctypes.c_double), ("mu", ctypes.c_double), ("iters", ctypes.c_int32),
                ("tag", ctypes.c_uint64), ("flags", ctypes.c_uint32), ("delta", ctypes.c_double),
                ("far", ctypes.c_void_p)]


class Far(ctypes.Structure):
    """stokes_far: the treecode's parameters for the u_bar sums of the solvers."""
    _fields_ = [("degree", ctypes.c_int32), ("theta", ctypes.c_double), ("leaf_size", ctypes.c_int32)]


def _far(far):
    """None, or (degree, theta[, leaf_size]) -> a Far by reference."""
    if far is None:
        return None
    deg, theta = far[0], far[1]
    leaf = far[2] if len(far) > 2 else 0
    return ctypes.byref(Far(int(deg), float(theta), int(leaf)))


class SolveStats(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_finish_ns", ctypes.c_int64), ("iters", ctypes.c_int32),
                ("status", ctypes.c_int32), ("residual", ctypes.c_double),
                ("tag", ctypes.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libstokes.so not built ({LIB_PATH}); run __graft_entry__.build() "
                          "or python paper_1602_05650_amd/csrc/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                           ctypes.c_double)
    sig = {
        "stokes_sl_eval": [I64, P, P, P, P, I32, P, I64, P, P, P, D, D, D, U32, P, P, P],
        "stokes_sl_eval_noalloc": [I64, P, P, P, P, I32, P, I64, P, P, P, D, D, D, U32, P, P],
        "stokes_dl_eval": [I64, P, P, P, P, I64, P, P, D, U32, P, P, P],
        "stokes_local_sbt": [I64, P, P, D, D, ctypes.c_int, P, P],
        "stokes_mobility_solve": [I32, I32, P, P, P, P, D, D, D, I32, U32, P, P, P, P, P],
        "stokes_nonlocal_sbt": [I32, I32, P, P, P, P, D, D, P, P],
        "stokes_tree_create": [I64, P, I64, P, I32, D, I32, P, P],
        "stokes_tree_sl_eval": [P, P, P, P, I32, P, D, D, D, U32, P, P],
        "stokes_tree_dl_eval": [P, P, P, P, D, U32, P, P],
        "stokes_tree_info": [P, P, P, P, P],
        "stokes_tree_destroy": [P],
        "stokes_particle_solve": [I64, P, P, P, I32, P, P, P, P, P, P, P, D, D, I32, U32, P, P, P,
                                  P, P, P],
        "stokes_fiber_step": [I32, I32, P, P, P, P, D, D, D, D, D, D, I32, D, U32, P, P, P, P, P, P],
        "stokes_session_create": [P, P],
        "stokes_session_submit": [P, P, P],
        "stokes_session_wait": [P, ctypes.c_uint64, P, P, I32],
        "stokes_session_cancel": [P, ctypes.c_uint64],
        "stokes_session_inject_fault": [P],
        "stokes_session_destroy": [P],
        "stokes_release_workspace": [],
        "stokes_version": [],
        "stokes_profile_enable": [ctypes.c_int],
        "stokes_profile_read": [P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.stokes_solve_footprint.argtypes = [I32, I32, I32, U32]
    lib.stokes_solve_footprint.restype = ctypes.c_int64
    lib.stokes_status_string.argtypes = [ctypes.c_int]
    lib.stokes_status_string.restype = ctypes.c_char_p
    lib.stokes_last_error.argtypes = []
    lib.stokes_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def status_string(code: int) -> str:
    return _lib.stokes_status_string(int(code)).decode()


def last_error() -> str:
    return _lib.stokes_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise StokesError(rc, last_error())


def _dev(t: Optional[torch.Tensor], dtype, name, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch tensor on a GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def sl_eval(src_xyz, src_force, *, src_weight=None, src_fiber=None, fiber_len=None, n_fib=None,
            trg_xyz=None, trg_self=None, trg_fiber=None, mu=1.0, eps=0.01, near_r=0.0,
            mixed=False, excl="self", doublet=True, accumulate=False, out=None,
            check_inputs=False, diag=False, stream=None):
    """Single-layer (Stokeslet + doublet) sum; returns (3, n_trg) float64 [, Diag].

    With src_fiber given, the fiber count is fiber_len's length, or n_fib."""
    src_xyz = _dev(src_xyz, torch.float64, "src_xyz")
    ns = src_xyz.shape[1]
    _dev(src_force, torch.float64, "src_force", (3, ns))
    _dev(src_weight, torch.float64, "src_weight", (ns,))
    _dev(src_fiber, torch.int32, "src_fiber", (ns,))
    _dev(fiber_len, torch.float64, "fiber_len")
    _dev(trg_xyz, torch.float64, "trg_xyz")
    nt = ns if trg_xyz is None else trg_xyz.shape[1]
    _dev(trg_self, torch.int64, "trg_self", (nt,))
    _dev(trg_fiber, torch.int32, "trg_fiber", (nt,))
    if out is None:
        out = (torch.zeros if accumulate else torch.empty)((3, nt), dtype=torch.float64,
                                                           device=src_xyz.device)
    _dev(out, torch.float64, "out", (3, nt))
    if nt == 0:          # an empty tensor has no data pointer, and NULL targets mean "the sources"
        return (out, Diag()) if diag else out
    flags = PREC_MIXED if mixed else PREC_FP64
    flags |= {"self": EXCL_SELF_POINT, "fiber": EXCL_SAME_FIBER, None: 0, "none": 0}[excl]
    flags |= 0 if doublet else NO_DOUBLET
    flags |= ACCUMULATE if accumulate else 0
    flags |= CHECK_INPUTS if check_inputs else 0
    if src_fiber is None:
        n_fib = 0
    elif fiber_len is not None:
        n_fib = fiber_len.shape[0]
    elif n_fib is None:
        raise ValueError("src_fiber given: pass fiber_len or n_fib")
    d = Diag() if diag else None
    rc = _lib.stokes_sl_eval(ns, _ptr(src_xyz), _ptr(src_force), _ptr(src_weight),
                             _ptr(src_fiber), n_fib, _ptr(fiber_len), nt, _ptr(trg_xyz),
                             _ptr(trg_self), _ptr(trg_fiber), float(mu), float(eps),
                             float(near_r), flags, _ptr(out), _stream(stream),
                             ctypes.byref(d) if d is not None else None)
    _check(rc)
    return (out, d) if diag else out


def sl_eval_noalloc(src_xyz, src_force, *, src_weight=None, src_fiber=None, fiber_len=None,
                    n_fib=None, trg_xyz=None, trg_self=None, trg_fiber=None, mu=1.0, eps=0.01,
                    near_r=0.0, mixed=False, excl="self", doublet=True, accumulate=False, out=None,
                    stream=None):
    """sl_eval through the entry point that allocates nothing (the library's static
    per-GPU scratch; no diagnostics, no input scan).  `out` (3, n_trg) float64 on the
    device is allocated here when not given, as for sl_eval."""
    src_xyz = _dev(src_xyz, torch.float64, "src_xyz")
    ns = src_xyz.shape[1]
    _dev(src_force, torch.float64, "src_force", (3, ns))
    _dev(src_weight, torch.float64, "src_weight", (ns,))
    _dev(src_fiber, torch.int32, "src_fiber", (ns,))
    _dev(fiber_len, torch.float64, "fiber_len")
    _dev(trg_xyz, torch.float64, "trg_xyz")
    nt = ns if trg_xyz is None else trg_xyz.shape[1]
    _dev(trg_self, torch.int64, "trg_self", (nt,))
    _dev(trg_fiber, torch.int32, "trg_fiber", (nt,))
    if out is None:
        out = (torch.zeros if accumulate else torch.empty)((3, nt), dtype=torch.float64,
                                                           device=src_xyz.device)
    _dev(out, torch.float64, "out", (3, nt))
    if nt == 0:
        return out
    flags = PREC_MIXED if mixed else PREC_FP64
    flags |= {"self": EXCL_SELF_POINT, "fiber": EXCL_SAME_FIBER, None: 0, "none": 0}[excl]
    flags |= 0 if doublet else NO_DOUBLET
    flags |= ACCUMULATE if accumulate else 0
    if src_fiber is None:
        n_fib = 0
    elif fiber_len is not None:
        n_fib = fiber_len.shape[0]
    elif n_fib is None:
        raise ValueError("src_fiber given: pass fiber_len or n_fib")
    rc = _lib.stokes_sl_eval_noalloc(ns, _ptr(src_xyz), _ptr(src_force), _ptr(src_weight),
                                     _ptr(src_fiber), n_fib, _ptr(fiber_len), nt, _ptr(trg_xyz),
                                     _ptr(trg_self), _ptr(trg_fiber), float(mu), float(eps),
                                     float(near_r), flags, _ptr(out), _stream(stream))
    _check(rc)
    return out


def dl_eval(src_xyz, src_normal, src_weight, src_q, *, trg_xyz=None, trg_self=None,
            near_r=0.0, mixed=False, subtract=True, accumulate=False, out=None,
            check_inputs=False, diag=False, stream=None):
    """Double-layer (stresslet) sum; returns (3, n_trg) float64 [, Diag]."""
    src_xyz = _dev(src_xyz, torch.float64, "src_xyz")
    ns = src_xyz.shape[1]
    _dev(src_normal, torch.float64, "src_normal", (3, ns))
    _dev(src_weight, torch.float64, "src_weight", (ns,))
    _dev(src_q, torch.float64, "src_q", (3, ns))
    _dev(trg_xyz, torch.float64, "trg_xyz")
    nt = ns if trg_xyz is None else trg_xyz.shape[1]
    _dev(trg_self, torch.int64, "trg_self", (nt,))
    if out is None:
        out = (torch.zeros if accumulate else torch.empty)((3, nt), dtype=torch.float64,
                                                           device=src_xyz.device)
    _dev(out, torch.float64, "out", (3, nt))
    if nt == 0:
        return (out, Diag()) if diag else out
    flags = (PREC_MIXED if mixed else PREC_FP64) | (0 if subtract else ONSURF_RAW)
    flags |= ACCUMULATE if accumulate else 0
    flags |= CHECK_INPUTS if check_inputs else 0
    d = Diag() if diag else None
    rc = _lib.stokes_dl_eval(ns, _ptr(src_xyz), _ptr(src_normal), _ptr(src_weight), _ptr(src_q),
                             nt, _ptr(trg_xyz), _ptr(trg_self), float(near_r), flags, _ptr(out),
                             _stream(stream), ctypes.byref(d) if d is not None else None)
    _check(rc)
    return (out, d) if diag else out


def local_sbt(tangent, f, eps, mu=1.0, inverse=False, out=None, stream=None):
    """Local slender-body operator M f (or M^{-1} f) at every node, (3, n) float64."""
    tangent = _dev(tangent, torch.float64, "tangent")
    n = tangent.shape[1]
    _dev(f, torch.float64, "f", (3, n))
    if out is None:
        out = torch.empty_like(f)
    _dev(out, torch.float64, "out", (3, n))
    _check(_lib.stokes_local_sbt(n, _ptr(tangent), _ptr(f), float(eps), float(mu),
                                 1 if inverse else 0, _ptr(out), _stream(stream)))
    return out


def _solve_opts(delta, precond):
    if precond not in ("local", "block"):
        raise ValueError(f"precond must be 'local' or 'block', not {precond!r}")
    return ((NONLOCAL if delta is not None else 0) | (PRECOND_BLOCK if precond == "block" else 0),
            0.0 if delta is None else float(delta))


def nonlocal_sbt(xyz, tangent, fiber_len, f, nodes_per_fib, delta, mu=1.0, out=None, stream=None):
    """K_delta[f] (regularised nonlocal slender-body self term) at every node, (3, N) float64."""
    xyz = _dev(xyz, torch.float64, "xyz")
    n = xyz.shape[1]
    _dev(tangent, torch.float64, "tangent", (3, n))
    _dev(fiber_len, torch.float64, "fiber_len")
    _dev(f, torch.float64, "f", (3, n))
    if out is None:
        out = torch.empty_like(f)
    _dev(out, torch.float64, "out", (3, n))
    _check(_lib.stokes_nonlocal_sbt(fiber_len.shape[0], int(nodes_per_fib), _ptr(xyz),
                                    _ptr(tangent), _ptr(fiber_len), _ptr(f), float(delta),
                                    float(mu), _ptr(out), _stream(stream)))
    return out


def mobility_solve(xyz, tangent, fiber_len, rhs, nodes_per_fib, eps, iters, mu=1.0, mixed=False,
                   doublet=True, delta=None, precond="local", far=None, stream=None):
    """GMRES mobility solve on device tensors; returns (f, residual, iterations).
    delta given: the operator includes the nonlocal self term K_delta; precond "block"
    uses each fiber's inverted self block instead of the local 3x3 blocks; far =
    (degree, theta[, leaf_size]): the other fibers' flow through a treecode plan."""
    xyz = _dev(xyz, torch.float64, "xyz")
    n = xyz.shape[1]
    _dev(tangent, torch.float64, "tangent", (3, n))
    _dev(fiber_len, torch.float64, "fiber_len")
    _dev(rhs, torch.float64, "rhs", (3, n))
    n_fib = fiber_len.shape[0]
    out = torch.empty_like(rhs)
    res = ctypes.c_double(0.0)
    it = ctypes.c_int32(0)
    opts, dl = _solve_opts(delta, precond)
    flags = (PREC_MIXED if mixed else PREC_FP64) | (0 if doublet else NO_DOUBLET) | opts
    _check(_lib.stokes_mobility_solve(n_fib, nodes_per_fib, _ptr(xyz), _ptr(tangent),
                                      _ptr(fiber_len), _ptr(rhs), float(eps), float(mu), dl,
                                      int(iters), flags, _ptr(out), ctypes.byref(res),
                                      ctypes.byref(it), _far(far), _stream(stream)))
    return out, res.value, it.value


class ParticleGeometry:
    """The surfaces of a particle solve packed on the device once: the particles'
    points, outward normals and weights concatenated as planes (particle p at
    offsets[p]..offsets[p + 1]), their centres, and the periphery's arrays (or none).

    particles: list of (xyz (3, M), outward normals (3, M), weights (M,), centre (3,));
    periphery: (xyz, outward normals, weights) or None for an unbounded fluid.  Arrays
    may be numpy or torch."""

    def __init__(self, particles, periphery=None):
        import numpy as np
        dev = torch.device("cuda", torch.cuda.current_device())

        def d(a):
            if isinstance(a, torch.Tensor):
                return a.to(device=dev, dtype=torch.float64).contiguous()
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

        def host(a):
            return a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else np.asarray(a, np.float64)

        self.device = dev
        self.n_part = len(particles)
        sizes = [host(pt[0]).shape[1] for pt in particles]
        self.offsets = (ctypes.c_int64 * (self.n_part + 1))(
            *np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64))
        self.yp = d(np.concatenate([host(pt[0]) for pt in particles], axis=1))
        self.np = d(np.concatenate([host(pt[1]) for pt in particles], axis=1))
        self.wp = d(np.concatenate([host(pt[2]) for pt in particles]))
        self.centres = d(np.stack([host(pt[3]) for pt in particles], axis=1))
        if periphery is None:
            self.m0, self.y0, self.n0, self.w0 = 0, None, None, None
        else:
            self.y0, self.n0, self.w0 = (d(a) for a in periphery)
            self.m0 = self.y0.shape[1]
        self.ms = self.m0 + int(sum(sizes))


def particle_solve(particles, force, torque, periphery=None, mu=1.0, iters=40, mixed=False,
                   near_r=0.0, eager=False, stream=None):
    """Mobility of rigid particles in a fixed periphery (second-kind boundary integrals).

    particles: a ParticleGeometry, or the list it is made from (with periphery:
    (xyz, outward normals, weights) or None for an unbounded fluid; ignored with a
    ParticleGeometry); force, torque: (3, n_particles), numpy or torch (copied to the
    device unless they are float64 device tensors already).  eager: launch each
    iteration's kernels one by one instead of replaying a captured graph.  Returns
    (U (3, n_p), Omega (3, n_p), q (3, M_s) device tensors, residual, iterations)."""
    import numpy as np
    g = particles if isinstance(particles, ParticleGeometry) else ParticleGeometry(particles, periphery)
    dev = g.device

    def d(a):
        if isinstance(a, torch.Tensor):
            return a.to(device=dev, dtype=torch.float64).contiguous()
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    n_p = g.n_part
    F, L = d(force).reshape(3, n_p), d(torque).reshape(3, n_p)
    U = torch.empty((3, n_p), dtype=torch.float64, device=dev)
    Om = torch.empty_like(U)
    q = torch.empty((3, g.ms), dtype=torch.float64, device=dev)
    res = ctypes.c_double(0.0)
    it = ctypes.c_int32(0)
    nz = lambda t: None if t is None else _ptr(t)
    _check(_lib.stokes_particle_solve(g.m0, nz(g.y0), nz(g.n0), nz(g.w0), n_p, g.offsets, _ptr(g.yp),
                                      _ptr(g.np), _ptr(g.wp), _ptr(g.centres), _ptr(F), _ptr(L), float(mu),
                                      float(near_r), int(iters),
                                      (PREC_MIXED if mixed else PREC_FP64) | (EAGER if eager else 0),
                                      _ptr(U), _ptr(Om), _ptr(q), ctypes.byref(res), ctypes.byref(it),
                                      _stream(stream)))
    return U, Om, q, res.value, it.value


def fiber_step(xyz, fiber_len, f_ext, nodes_per_fib, eps, E, dt, mu=1.0, delta=None, iters=40,
               tol=0.0, mixed=False, doublet=True, near_r=0.0, clamp=None, far=None, stream=None):
    """One implicit (backward Euler) step of elastic fibers (stokes_fiber_step) on device
    tensors: xyz, f_ext (3, N), fiber_len (n_fib,).  delta given: the nonlocal self term
    K_delta is included.  clamp: (n_fib,) minus-end conditions at a body at rest
    (any array; 0 or False free, 1 or True clamped, 2 hinged).  far = (degree, theta[,
    leaf_size]): the other fibers' flow through a treecode plan of the step's nodes.
    Returns (X+ (3, N), T+ (N,), residual, iterations)."""
    xyz = _dev(xyz, torch.float64, "xyz")
    n = xyz.shape[1]
    _dev(fiber_len, torch.float64, "fiber_len")
    _dev(f_ext, torch.float64, "f_ext", (3, n))
    n_fib = fiber_len.shape[0]
    if n_fib * int(nodes_per_fib) != n:
        raise ValueError("fiber_len and nodes_per_fib do not match xyz")
    cl = None
    if clamp is not None:
        import numpy as np
        host = clamp.detach().cpu().numpy() if isinstance(clamp, torch.Tensor) else np.asarray(clamp)
        if host.size != n_fib:
            raise ValueError("clamp must have one flag per fiber")
        host = host.ravel().astype(np.int64)
        if np.any((host < 0) | (host > 2)):
            raise ValueError("clamp values must be 0 (free), 1 (clamped) or 2 (hinged)")
        cl = torch.from_numpy(host.astype(np.int32)).to(xyz.device)
    out = torch.empty_like(xyz)
    T = torch.empty((n,), dtype=torch.float64, device=xyz.device)
    res = ctypes.c_double(0.0)
    it = ctypes.c_int32(0)
    flags = ((PREC_MIXED if mixed else PREC_FP64) | (0 if doublet else NO_DOUBLET)
             | (NONLOCAL if delta is not None else 0))
    _check(_lib.stokes_fiber_step(n_fib, int(nodes_per_fib), _ptr(xyz), _ptr(fiber_len), _ptr(f_ext),
                                  None if cl is None else _ptr(cl), float(eps), float(E), float(dt), float(mu),
                                  float(delta) if delta is not None else 0.0, float(near_r), int(iters),
                                  float(tol), flags, _ptr(out), _ptr(T), ctypes.byref(res),
                                  ctypes.byref(it), _far(far), _stream(stream)))
    return out, T, res.value, it.value


class Tree:
    """Treecode plan for the single-layer sum over fixed source and target positions
    (device tensors); see stokes_tree_create."""

    def __init__(self, src_xyz, trg_xyz=None, degree=6, theta=0.7, leaf_size=128, stream=None):
        self._src = _dev(src_xyz, torch.float64, "src_xyz")
        self.n_src = self._src.shape[1]
        if trg_xyz is not None:
            trg_xyz = _dev(trg_xyz, torch.float64, "trg_xyz")
        self.n_trg = self.n_src if trg_xyz is None else trg_xyz.shape[1]
        self._h = ctypes.c_void_p()
        _check(_lib.stokes_tree_create(self.n_src, _ptr(self._src), self.n_trg,
                                       None if trg_xyz is None else _ptr(trg_xyz), int(degree),
                                       float(theta), int(leaf_size), _stream(stream),
                                       ctypes.byref(self._h)))

    def sl_eval(self, force, src_fiber=None, fiber_len=None, src_weight=None, mu=1.0, eps=0.01,
                near_r=0.0, excl_self=True, mixed=False, doublet=True, out=None, accumulate=False,
                stream=None, excl_fiber=False, check_inputs=False):
        """excl_fiber: skip every source of the target's fiber (plans with targets = sources;
        needs src_fiber) instead of only the target's own point.  check_inputs: the input
        scan of sl_eval (synchronous)."""
        _dev(force, torch.float64, "force", (3, self.n_src))
        if src_fiber is not None:
            _dev(src_fiber, torch.int32, "src_fiber", (self.n_src,))
            _dev(fiber_len, torch.float64, "fiber_len")
        if src_weight is not None:
            _dev(src_weight, torch.float64, "src_weight", (self.n_src,))
        if out is None:
            out = torch.zeros((3, self.n_trg), dtype=torch.float64, device=force.device)
        excl = EXCL_SAME_FIBER if excl_fiber else (EXCL_SELF_POINT if excl_self else 0)
        flags = ((PREC_MIXED if mixed else PREC_FP64) | excl
                 | (0 if doublet else NO_DOUBLET) | (ACCUMULATE if accumulate else 0)
                 | (CHECK_INPUTS if check_inputs else 0))
        nz = lambda t: None if t is None else _ptr(t)
        n_fib = 0 if fiber_len is None else fiber_len.shape[0]
        _check(_lib.stokes_tree_sl_eval(self._h, _ptr(force), nz(src_weight), nz(src_fiber), n_fib,
                                        nz(fiber_len), float(mu), float(eps), float(near_r), flags,
                                        _ptr(out), _stream(stream)))
        return out

    def dl_eval(self, normal, weight, q, raw=False, out=None, accumulate=False, stream=None, mixed=False,
                near_r=0.0):
        """Double-layer sum of dl_eval on this plan (FP64, or mixed: FP32 pairs with FP64
        pairs closer than near_r, <= 0 selecting 0.02).  Plans built with targets =
        sources take the singularity subtraction unless raw."""
        _dev(normal, torch.float64, "normal", (3, self.n_src))
        _dev(weight, torch.float64, "weight", (self.n_src,))
        _dev(q, torch.float64, "q", (3, self.n_src))
        if out is None:
            out = torch.zeros((3, self.n_trg), dtype=torch.float64, device=q.device)
        flags = ((PREC_MIXED if mixed else PREC_FP64) | (ONSURF_RAW if raw else 0)
                 | (ACCUMULATE if accumulate else 0))
        _check(_lib.stokes_tree_dl_eval(self._h, _ptr(normal), _ptr(weight), _ptr(q), float(near_r), flags,
                                        _ptr(out), _stream(stream)))
        return out

    def info(self):
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        c, d = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.stokes_tree_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                     ctypes.byref(d)))
        return {"proxy_pairs": a.value, "direct_pairs": b.value, "proxy_clusters": c.value,
                "batches": d.value}

    def close(self):
        if self._h:
            h, self._h = self._h, None
            _check(_lib.stokes_tree_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on=True):
    """Bracket every launch of the main pair-sum kernels with HIP events (on the call's stream)."""
    _check(_lib.stokes_profile_enable(1 if on else 0))


def profile_read():
    """(milliseconds, launches) of the main pair-sum kernels since the last read; resets."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(_lib.stokes_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def solve_footprint(n_fib, nodes_per_fib, iters, mixed=False, precond="local"):
    """Device bytes a mobility request of this shape takes from a session budget."""
    flags = (PREC_MIXED if mixed else PREC_FP64) | (PRECOND_BLOCK if precond == "block" else 0)
    return int(_lib.stokes_solve_footprint(int(n_fib), int(nodes_per_fib), int(iters), flags))


def release_workspace():
    _check(_lib.stokes_release_workspace())


def version() -> int:
    return _lib.stokes_version()


class Session:
    """Continuous-batching mobility-solve session (host arrays in, host arrays out)."""

    def __init__(self, hbm_budget_bytes=4 << 30, max_slots=64, max_queue=4096, mixed=False,
                 doublet=True, device=0, step_pairs=0):
        """step_pairs: single-layer pairs one request may take per step (0: the
        library default, < 0: a whole matvec per step)."""
        cfg = SessionCfg(int(hbm_budget_bytes), int(max_slots), int(max_queue),
                         (PREC_MIXED if mixed else PREC_FP64) | (0 if doublet else NO_DOUBLET),
                         int(device), int(step_pairs))
        self._h = ctypes.c_void_p()
        _check(_lib.stokes_session_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._shapes = {}

    def submit(self, xyz, tangent, fiber_len, rhs, nodes_per_fib, eps, iters, mu=1.0, tag=0,
               delta=None, precond="local", far=None):
        """far = (degree, theta[, leaf_size]): the request's u_bar sums through a treecode
        plan of its nodes (built at admission)."""
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (xyz, tangent, fiber_len, rhs)]
        n = arrs[0].shape[1]
        opts, dl = _solve_opts(delta, precond)
        farp = None
        if far is not None:
            farp = Far(int(far[0]), float(far[1]), int(far[2]) if len(far) > 2 else 0)
        req = SolveReq(int(arrs[2].shape[0]), int(nodes_per_fib),
                       arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                       arrs[3].ctypes.data, float(eps), float(mu), int(iters), int(tag),
                       opts, dl, ctypes.addressof(farp) if farp is not None else None)
        t = ctypes.c_uint64(0)
        _check(_lib.stokes_session_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._shapes[t.value] = n
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        """Returns (f (3, N) numpy, stats dict); raises StokesError on failure."""
        import numpy as np
        n = self._shapes.get(ticket, 0)
        out = np.empty((3, n), dtype=np.float64)
        st = SolveStats()
        rc = _lib.stokes_session_wait(self._h, ctypes.c_uint64(ticket),
                                      out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st),
                                      int(timeout_ms))
        if rc not in (E_TIMEOUT, E_BUSY):      # the ticket is still live after these
            self._shapes.pop(ticket, None)
        _check(rc)
        stats = {f: getattr(st, f) for f, _ in SolveStats._fields_}
        return out, stats

    def inject_fault(self):
        """Test hook: the next step fails every request then in flight."""
        _check(_lib.stokes_session_inject_fault(self._h))

    def cancel(self, ticket):
        _check(_lib.stokes_session_cancel(self._h, ctypes.c_uint64(ticket)))

    def close(self):
        if self._h:
            h, self._h = self._h, None
            _check(_lib.stokes_session_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
