"""MI355X-native nodal discontinuous Galerkin Runge-Kutta stepping.

The compute path is the HIP library ``libdg.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/dg.h``; ``dg`` is its thin ctypes binding and
``workloads`` the seeded synthetic inputs. Importing this package loads
nothing; the binding loads the library on first use and raises if it is
missing.
"""
__all__ = ["dg", "workloads"]
