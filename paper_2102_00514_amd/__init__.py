"""Parallel-in-time iterated extended / sigma-point Kalman smoother for MI355X (gfx950).

* ``binding``   -- ctypes binding of the HIP library ``libsmoother.so`` (include/smoother.h)
* ``workloads`` -- seeded synthetic problem instances (coordinated turn + bearings, linear)
* ``build``     -- builds the HIP library with hipcc
"""
__all__ = ["binding", "workloads", "build"]
__version__ = "0.1.0"
