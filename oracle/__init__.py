"""Plain, slow, FP64 CPU oracle for the p2o map and the data-space inversion.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library
and its Python binding) never does, and shares no code with it.
"""
from .p2o_oracle import *  # noqa: F401,F403
