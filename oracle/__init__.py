"""FP64 CPU oracle of the halfway-domain scene-flow solve.

Test infrastructure only: imported by the tests, the smoke entry point and
the benchmark's CPU-baseline leg, never by the library."""
from .halfway import *  # noqa: F401,F403
