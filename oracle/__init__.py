"""FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the GPU library never does, and this package imports
nothing from it.
"""
from .nuasm_oracle import *  # noqa: F401,F403
from .nuasm_oracle import __all__  # noqa: F401
