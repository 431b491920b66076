"""Plain FP64 CPU oracle of the anti-lopsided NNLS method.

Test infrastructure only: the test suite, the smoke check and the benchmark's CPU-baseline leg
use it to judge the HIP library.  The product package never imports it.
"""
from .oracle import *  # noqa: F401,F403
