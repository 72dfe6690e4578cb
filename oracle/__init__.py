"""FP64 CPU oracle for polynomial-preconditioned FISTA (TEST INFRASTRUCTURE ONLY).

This package is the plain, slow, obviously-correct statement of what the GPU
library computes, written from the paper (Iyer et al., "Polynomial
Preconditioners for Regularized Linear Inverse Problems", arXiv 2204.10252).
It shares no code with the GPU path and must only be imported by the test
suite, by ``__graft_entry__.smoke()`` and by the CPU-baseline leg of
``bench.py``.  Nothing in the product library may call it.

Pinned: every function here is checked in ``tests/test_oracle_*.py`` against
closed forms, theorems of the paper, textbook definitions or brute force
(finite differences for the derivatives of ``pfista_vjp``).
"""

from .pfista_oracle import *  # noqa: F401,F403
from .pfista_oracle import __all__ as _ops_all
from .pfista_toeplitz import *  # noqa: F401,F403
from .pfista_toeplitz import __all__ as _toe_all
from .pfista_vjp import *  # noqa: F401,F403
from .pfista_vjp import __all__ as _vjp_all

__all__ = list(_ops_all) + list(_vjp_all) + list(_toe_all)
