"""FP64 CPU oracle of the LAKER solve path.  TEST INFRASTRUCTURE ONLY: imported by
tests, the smoke check and the benchmark's CPU-baseline leg, never by the library."""
from . import laker_oracle, learned_oracle  # noqa: F401
