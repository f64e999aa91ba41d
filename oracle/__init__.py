"""Independent FP64 CPU oracle for the sheared model-H time step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check and
the benchmark's CPU-baseline leg may import this package.  The GPU library and
its Python binding never import it, and it imports nothing from them.
"""
from . import model_h, observables, scales  # noqa: F401
