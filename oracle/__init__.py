"""CPU FP64 oracle of the F-statistic search path.

TEST INFRASTRUCTURE ONLY.  This package exists to check the GPU library: it
may be imported by the tests, by the smoke check and by the CPU-baseline leg
of the benchmark, and by nothing else.  It shares no code with the GPU path.
"""
from .fstat_oracle import *  # noqa: F401,F403
