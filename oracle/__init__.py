"""CPU oracle for the Speed-ANN search path (arXiv 2201.13007).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU
baseline leg of the benchmark, never by the GPU library.  The arithmetic lives in
``oracle.c`` (plain C, gcc); this module compiles it, marshals numpy arrays and adds
the recall definition (Sec. 2.1, Eq. for Recall).
"""
from .oracle import *  # noqa: F401,F403
