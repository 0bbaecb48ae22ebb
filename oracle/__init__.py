"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The HIP library never calls it.
"""

from .oracle import Oracle, build_oracle, sector_counts  # noqa: F401
