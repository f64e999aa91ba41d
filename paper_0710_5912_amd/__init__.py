"""MI355X-native sheared model-H time step (2D Cahn-Hilliard + Navier-Stokes).

The compute path is the HIP library built from ``csrc/`` and reached through
the C ABI declared in ``include/le.h``; :mod:`paper_0710_5912_amd.le` is its
thin ctypes binding.  Importing this package loads nothing: the binding loads
the shared library on first use and raises if it is missing.
"""

__all__ = ["inputs", "configs"]
