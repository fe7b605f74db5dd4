"""CPU oracle for Rosko packing, SpMM, backward and the scheduler MLP.

Test infrastructure only: the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  The product path never imports it.
"""
from .oracle import *  # noqa: F401,F403
