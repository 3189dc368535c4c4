"""FP64 CPU oracle for the TACAW spectral reduction.

TEST INFRASTRUCTURE ONLY. Nothing in the product package may import, call or
execute anything in this directory; only the test suite, the smoke check and
the CPU-baseline leg of the benchmark use it. It shares no code, constants or
tables with the GPU library: it is written from the paper's statement of the
method (Eq. 1, the Welch chunking and windowing of Sec. II.B, the chunk average
of Eq. 2 and the detector integration of the DetectorSet description) in plain
NumPy float64/complex128.

Parity status per function is listed in ``tacaw_oracle.__doc__``.
"""

from .tacaw_oracle import *  # noqa: F401,F403
from .tacaw_oracle import __all__  # noqa: F401
