"""Float64 CPU oracle of the compressor (test infrastructure only: imported by
the tests, the smoke check and the benchmark's CPU-baseline leg, never by the
library)."""
from .dmc_oracle import *  # noqa: F401,F403
