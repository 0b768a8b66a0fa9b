"""FP64 CPU oracle for the NOLSM hot path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  The library never does.
"""
from . import nolsm_oracle  # noqa: F401
