"""FP64 CPU oracle for butterfly filtering -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this package.
"""
from . import bfly_oracle  # noqa: F401
