"""FP64 CPU oracle for the fast-resolve response operator.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's cpu_baseline leg, never by the product path.  It shares no code with
the HIP library (paper_2406_09144_amd); the two meet only in the seeded input
generators of the `synthetic` package.

Every function states the passage of the paper it writes out.  The direct sums
live in dft.c (plain C, OpenMP), the rest in reference.py (numpy, float64).
"""

from .reference import *  # noqa: F401,F403
from .build import build, lib_path  # noqa: F401
