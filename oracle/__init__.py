"""FP64 CPU oracle of the uplink receiver (fft -> csi -> equal -> demod).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
the benchmark's CPU-baseline leg may import it.  The product path never calls
it and shares no code with it.
"""
from .rxphy_oracle import *  # noqa: F401,F403
from . import sensing_oracle  # noqa: F401,E402
