"""FP64 CPU oracle for the TLMPM cutting hot path.

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg of the
benchmark load it.  The product library never imports it.
"""
from .oracle import *  # noqa: F401,F403
