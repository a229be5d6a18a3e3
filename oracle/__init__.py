"""FP64 CPU oracle for the BSE eigenproblem (forms I and II) -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP solver.
"""
from .bse import *  # noqa: F401,F403
from . import metrics  # noqa: F401
