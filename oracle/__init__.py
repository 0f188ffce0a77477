"""FP64 CPU oracle of the FGA hot path (arXiv 2009.14005).

TEST INFRASTRUCTURE ONLY: this package is the plain, slow reference that the
HIP path is checked against. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the product library never does,
and the two share no code.

Parity pins: every function here is pinned by ``tests/test_oracle_pins.py``
against closed forms, brute force in extended precision, invariants or a
library routine (see the module docstrings of ``oracle.core``).
"""
from .core import *  # noqa: F401,F403
from .core import __all__  # noqa: F401
