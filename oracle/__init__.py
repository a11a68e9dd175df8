"""FP64 CPU oracle for the ladder (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never links or calls it.  It shares no
code with the HIP path: the C source is compiled with gcc on its own, and the only
module both sides use is ``synthetic`` (counter-based random draws, no ladder
arithmetic).
"""
from .oracle import *  # noqa: F401,F403
