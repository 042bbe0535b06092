"""MI355X-native free-space Stokes kernel sums for slender-body fiber suspensions.

The compute path is the HIP library ``libstokes.so`` (C ABI declared in
``include/stokes.h``); ``paper_1602_05650_amd.stokes`` is its thin ctypes
binding (importing it loads the library and fails loudly if it is missing).
``paper_1602_05650_amd.workloads`` holds the seeded synthetic geometries.
Submodules are imported on demand, so the generators need no GPU library.
"""
