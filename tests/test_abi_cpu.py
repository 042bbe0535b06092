"""The C-ABI library loads and exports every entry point the header declares.

CPU only: loading libstokes.so does not touch a GPU, and argument validation
returns before any device call, so the status contract is checked here too.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stokes.h")
LIB = os.path.join(ROOT, "paper_1602_05650_amd", "libstokes.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(stokes_\w+)\s*\(", text, re.M)))


def test_header_declares_required_entry_points():
    names = declared()
    for req in ["stokes_sl_eval", "stokes_dl_eval", "stokes_session_submit", "stokes_session_create",
                "stokes_session_wait", "stokes_session_cancel", "stokes_session_destroy",
                "stokes_status_string", "stokes_local_sbt", "stokes_mobility_solve"]:
        assert req in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_status_strings_and_validation_without_gpu():
    from paper_1602_05650_amd import stokes as S
    assert S.status_string(S.OK) == "STOKES_OK"
    assert S.status_string(S.E_NONFINITE) == "STOKES_E_NONFINITE"
    assert S.status_string(99) == "STOKES_E_UNKNOWN"
    L = S._lib
    # n_src < 0
    assert L.stokes_sl_eval(-1, None, None, None, None, 0, None, 0, None, None, None,
                            1.0, 0.01, 0.0, 0, None, None, None) == S.E_INVAL
    assert "n_src" in S.last_error()
    # eps outside (0, 0.5)
    assert L.stokes_sl_eval(0, None, None, None, None, 0, None, 0, None, None, None,
                            1.0, 0.7, 0.0, 0, None, None, None) == S.E_INVAL
    # mu <= 0
    assert L.stokes_sl_eval(0, None, None, None, None, 0, None, 0, None, None, None,
                            0.0, 0.01, 0.0, 0, None, None, None) == S.E_INVAL
    # both exclusion modes
    assert L.stokes_sl_eval(0, None, None, None, None, 0, None, 0, None, None, None, 1.0, 0.01,
                            0.0, S.EXCL_SELF_POINT | S.EXCL_SAME_FIBER, None, None, None) == S.E_INVAL
    # unknown flag bits
    assert L.stokes_dl_eval(0, None, None, None, None, 0, None, None, 0.0, 1 << 20, None, None,
                            None) == S.E_INVAL
    # null arrays with n > 0
    assert L.stokes_dl_eval(4, None, None, None, None, 0, None, None, 0.0, 0, None, None,
                            None) == S.E_INVAL
    # empty problems are fine and touch nothing
    assert L.stokes_sl_eval(0, None, None, None, None, 0, None, 0, ctypes.c_void_p(8), None, None,
                            1.0, 0.01, 0.0, 0, None, None, None) == S.OK
    assert L.stokes_local_sbt(0, None, None, 0.01, 1.0, 0, None, None) == S.OK
    assert L.stokes_local_sbt(3, None, None, 0.01, 1.0, 0, None, None) == S.E_INVAL
    assert L.stokes_mobility_solve(1, 1, None, None, None, None, 0.01, 1.0, 0.0, 5, 0, None,
                                   None, None, None, None) == S.E_INVAL
    assert L.stokes_mobility_solve(1, 8, None, None, None, None, 0.01, 1.0, 0.0, 0, 0, None,
                                   None, None, None, None) == S.E_INVAL
    # the nonlocal term needs delta > 0; unknown flag bits are refused
    assert L.stokes_mobility_solve(1, 8, None, None, None, None, 0.01, 1.0, 0.0, 5, S.NONLOCAL,
                                   None, None, None, None, None) == S.E_INVAL
    assert "delta" in S.last_error()
    assert L.stokes_mobility_solve(1, 8, None, None, None, None, 0.01, 1.0, 0.0, 5, 1 << 12,
                                   None, None, None, None, None) == S.E_INVAL
    # treecode far field: degree 1..10, theta in (0, 1), checked before any device work
    for deg, th in ((0, 0.5), (11, 0.5), (6, 0.0), (6, 1.0)):
        far = ctypes.byref(S.Far(deg, th, 0))
        assert L.stokes_mobility_solve(1, 8, None, None, None, None, 0.01, 1.0, 0.0, 5, 0,
                                       None, None, None, far, None) == S.E_INVAL
        assert "stokes_far" in S.last_error()
        assert L.stokes_fiber_step(0, 16, None, None, None, None, 0.01, 1.0, 1e-3, 1.0, 0.0, 0.0, 10,
                                   0.0, 0, None, None, None, None, far, None) == S.E_INVAL
    # the entry point that allocates nothing: no input scan, and the size limit
    assert L.stokes_sl_eval_noalloc(0, None, None, None, None, 0, None, 0, ctypes.c_void_p(8), None, None,
                                    1.0, 0.01, 0.0, 0, None, None) == S.OK
    assert L.stokes_sl_eval_noalloc(2, ctypes.c_void_p(8), ctypes.c_void_p(8), None, None, 0, None, 0,
                                    None, None, None, 1.0, 0.01, 0.0, S.CHECK_INPUTS, ctypes.c_void_p(8),
                                    None) == S.E_INVAL
    assert L.stokes_nonlocal_sbt(0, 8, None, None, None, None, 0.01, 1.0, None, None) == S.OK
    assert L.stokes_nonlocal_sbt(2, 8, None, None, None, None, 0.0, 1.0, None, None) == S.E_INVAL
    assert L.stokes_nonlocal_sbt(2, 65, None, None, None, None, 0.01, 1.0, None, None) == S.E_INVAL
    # particle solve: every particle needs >= 4 points, part_offset starts at 0
    offs = (ctypes.c_int64 * 2)(0, 3)
    assert L.stokes_particle_solve(0, None, None, None, 1, offs, None, None, None, None, None, None,
                                   1.0, 0.0, 5, 0, None, None, None, None, None, None) == S.E_INVAL
    offs = (ctypes.c_int64 * 2)(1, 9)
    assert L.stokes_particle_solve(0, None, None, None, 1, offs, None, None, None, None, None, None,
                                   1.0, 0.0, 5, 0, None, None, None, None, None, None) == S.E_INVAL
    offs = (ctypes.c_int64 * 2)(0, 9)
    assert L.stokes_particle_solve(0, None, None, None, 1, offs, None, None, None, None, None, None,
                                   1.0, 0.0, 5, 0, None, None, None, None, None, None) == S.E_INVAL
    assert "null" in S.last_error()
    # treecode plans: parameters are checked before any device work
    h = ctypes.c_void_p()
    assert L.stokes_tree_create(0, None, 0, None, 6, 0.7, 128, None, ctypes.byref(h)) == S.E_INVAL
    assert L.stokes_tree_create(10, ctypes.c_void_p(8), 0, None, 11, 0.7, 128, None,
                                ctypes.byref(h)) == S.E_INVAL
    assert L.stokes_tree_create(10, ctypes.c_void_p(8), 0, None, 6, 1.5, 128, None,
                                ctypes.byref(h)) == S.E_INVAL
    assert "theta" in S.last_error()
    assert L.stokes_tree_sl_eval(None, None, None, None, 0, None, 1.0, 0.01, 0.0, 0, None,
                                 None) == S.E_INVAL
    assert L.stokes_tree_dl_eval(None, None, None, None, 0.0, 0, None, None) == S.E_INVAL
    assert L.stokes_tree_destroy(None) == S.E_INVAL
    assert L.stokes_session_create(None, None) == S.E_INVAL
    assert L.stokes_session_destroy(None) == S.E_INVAL


def test_solve_footprint_without_gpu():
    from paper_1602_05650_amd import stokes as S
    small = S.solve_footprint(10, 16, 20)
    big = S.solve_footprint(2048, 64, 60)
    assert 0 < small < big
    assert S.solve_footprint(10, 16, 20, mixed=True) > small        # FP32 packs on top
    assert S.solve_footprint(0, 16, 20) == 0 and S.solve_footprint(10, 65, 20) == 0
    # the Krylov basis alone: (k+1) x 3N doubles
    assert big > 61 * 3 * 2048 * 64 * 8
    # block-Jacobi adds the inverted fiber blocks: (3 npf)^2 doubles per fiber
    assert S.solve_footprint(10, 16, 20, precond="block") - small >= 10 * 48 * 48 * 8


def test_version():
    from paper_1602_05650_amd import stokes as S
    assert S.version() >= 10000


def test_fiber_step_validation_without_gpu():
    from paper_1602_05650_amd import stokes as S
    L = S._lib

    def call(n_fib=0, npf=16, eps=0.01, E=1.0, dt=1e-3, mu=1.0, delta=0.0, iters=10, tol=0.0, flags=0,
             ptrs=None):
        p = ptrs if ptrs is not None else [None] * 5
        return L.stokes_fiber_step(n_fib, npf, p[0], p[1], p[2], None, eps, E, dt, mu, delta, 0.0, iters,
                                   tol, flags, p[3], p[4], None, None, None, None)

    assert call() == S.OK                                   # no fibers: nothing to do
    for kw in ({"npf": 5}, {"npf": 49}, {"n_fib": -1}, {"eps": 0.6}, {"E": -1.0}, {"dt": 0.0},
               {"mu": 0.0}, {"iters": 0}, {"iters": 129}, {"tol": -1.0},
               {"flags": S.NONLOCAL}, {"flags": S.EXCL_SELF_POINT}, {"dt": float("nan")}):
        assert call(**kw) == S.E_INVAL, kw
    assert "stokes_fiber_step" in S.last_error()
    assert call(n_fib=2) == S.E_INVAL                       # null arrays with fibers
    assert "null" in S.last_error()
    fake = ctypes.c_void_p(1)
    assert call(n_fib=2, ptrs=[fake, fake, fake, fake, fake]) == S.E_INVAL   # X+ aliases X
    assert "alias" in S.last_error()
