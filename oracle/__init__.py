"""CPU FP64 oracle for the overlapping-fragments method (OFM) hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path (the HIP library and its binding) never does.  It shares no code with
the GPU path: it has its own potential evaluation, its own sparse
finite-difference operators, its own pair enumeration and its own dense
linear algebra (numpy / scipy, float64).
"""

from .ofm_oracle import *  # noqa: F401,F403
