"""Plain FP64 CPU oracle for the Wilson-clover AMG solver (test infrastructure).

This package is the correctness reference for the HIP library and nothing else:
only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  The library never calls into it, and it shares no code, header,
table or helper with the HIP path; the two meet only through the seeded inputs
of the ``synthetic`` module.

Every function is written from the paper (Kanamori, Ishikawa, Matsufuru,
"Object-oriented implementation of algebraic multi-grid solver for lattice QCD
on SIMD architectures and GPU clusters", arXiv:2111.05012) and cites the
section / equation / listing it follows.  Where the paper is silent, the
reading taken is stated in the docstring.

Parity status of each function (what pins it, besides itself) is listed in the
module docstrings of ``oracle.dirac`` and ``oracle.amg``.
"""
from . import dirac, amg  # noqa: F401
