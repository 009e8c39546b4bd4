"""FP64 CPU oracle for the four-step learned-wavelet decode path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product (the HIP
library and its Python binding) never calls it and shares no code with it.

Parity pins: every function is checked in tests/test_oracle_*.py against
something other than itself (closed forms, a library routine, brute force,
high-precision arithmetic or an invariant the paper states).  The mixture-head
parameterisation and the sigma floor are readings where the paper is silent;
their formulas are pinned against library routines, their choice is not pinned
by the paper.
"""
from .wv_oracle import *  # noqa: F401,F403
from .rans_ref import rans_encode_ref, rans_decode_ref  # noqa: F401
