"""MI355X-native SPSTD engine (symplectic pseudospectral time-domain solver
of the time-dependent Schroedinger equation, arXiv:1805.03155).

The solver lives in ``libspstd.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/spstd.h``); ``spstd`` is its thin ctypes binding and
``workloads`` the seeded synthetic inputs.
"""
__all__ = ["spstd", "workloads"]
