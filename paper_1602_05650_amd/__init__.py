"""MI355X-native free-space Stokes kernel sums for slender-body fiber suspensions.

The compute path is the HIP library ``libstokes.so`` (C ABI declared in
``include/stokes.h``); ``paper_1602_05650_amd.stokes`` is its thin ctypes
binding.  ``workloads`` holds the seeded synthetic geometries.
"""
__all__ = ["stokes", "workloads"]


def __getattr__(name):
    if name == "stokes":
        from . import stokes as _s
        return _s
    if name == "workloads":
        from . import workloads as _w
        return _w
    raise AttributeError(name)
