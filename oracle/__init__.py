"""FP64 CPU oracle of the ideal-MHD patch advance (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it.
"""

from .oracle import *  # noqa: F401,F403
