"""FP64 CPU oracle of the incompressible Inertial Coupling Method step.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product path never does.
"""
from . import philox, icm  # noqa: F401
