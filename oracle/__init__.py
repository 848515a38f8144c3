"""FP64 CPU oracle for the one-step photo-switching optoacoustic reconstruction.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, links or
calls this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP library (the seeded
input generators live in the separate `synth` package, which holds none of
the method's arithmetic).

Every function follows a passage of arXiv 2510.23739 (cited per function) in
plain NumPy float64, with no blocking or fusion beyond what the definition
states.  Pins against things other than itself live in tests/test_oracle_*.py.
"""
from .core import *  # noqa: F401,F403
from .core import __all__  # noqa: F401
