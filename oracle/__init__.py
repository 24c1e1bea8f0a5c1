"""FP64 CPU oracle for the 3-D Laplace FMM.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark; never by the product library.
"""
from .oracle import *  # noqa: F401,F403
