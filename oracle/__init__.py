"""FP64 CPU oracle of the hybrid finite-volume reconstruction.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; only
the test suite, the smoke check and the benchmark's CPU-baseline leg use it.
It is written from the paper (arXiv 2510.25906, Sections 2.1-2.5) in plain
NumPy and shares no code, table or constant with the GPU library; the two
meet only through the seeded input generators.

Parity pins (tests/test_oracle_*.py) tie every function to something other
than itself: closed-form integrals, polynomial exactness, conservation,
convergence order, limiting special cases, textbook shock relations and
brute-force checks.
"""
from .reconstruction import OracleModel, basis_exponents  # noqa: F401
from . import flux, quadrature, geometry  # noqa: F401
