"""Plain FP64 CPU oracle of the ISDF path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import anything from this package.  The product library never calls it, and
it shares no code with the HIP path.
"""
from .isdf_oracle import *  # noqa: F401,F403
