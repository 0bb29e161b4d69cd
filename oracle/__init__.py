"""FP64 CPU oracle for the implicit CP-ALS time step (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (the HIP library and its Python binding)
never calls it.
"""
from .cpals_oracle import *  # noqa: F401,F403
