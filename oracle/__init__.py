"""FP64 CPU oracle for the density-matrix solver -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct NumPy implementations of what the GPU path
computes, each function citing the passage of the paper it follows.  Only the
test-suite, the smoke check and the benchmark's CPU-baseline leg may import
this package; the product path never does, and the oracle shares no code with
the HIP implementation.

Parity status per function is stated in ``oracle/sp2_oracle.py``.
"""

from .sp2_oracle import *  # noqa: F401,F403
from . import precision_emulation  # noqa: F401,E402
from . import lanczos  # noqa: F401,E402
from .lanczos import lanczos_bounds  # noqa: F401,E402
from . import xlbomd  # noqa: F401,E402
from . import canonical  # noqa: F401,E402
from . import accelerated  # noqa: F401,E402
