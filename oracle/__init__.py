"""FP64 CPU oracle of the holotomography gradient (test infrastructure only:
imported by the tests, the smoke check and the benchmark's CPU-baseline leg,
never by the product path)."""
from . import holo_oracle  # noqa: F401
