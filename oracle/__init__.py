"""FP64 CPU oracle for the preconditioned multigrid Landweber method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; it is used by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark.  It is a plain, slow, direct transcription
of what the paper's method computes (projector, back-projector,
preconditioners, restriction/prolongation, regularisers, Landweber / SIRT,
OS-EMTR, Algorithm 1) in float64, written to be checked against the paper by
eye.  It shares no code with the HIP path.

Parity status of each function is listed in its docstring; functions whose
results are not pinned to anything outside the oracle say "parity unpinned".
"""

from .core import *  # noqa: F401,F403
from .methods import *  # noqa: F401,F403
from . import cnn  # noqa: F401
