"""CPU FP64 oracle for commutator-free exponential time-propagators (CFETs).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
product path (the HIP library and its Python binding) never imports, links or
executes this package, and this package never imports the product path.

Modules:
  schemes  coefficient tables (rule R1), shifted Legendre polynomials,
           Gauss-Legendre nodes/weights and the g[i,m] of Sec. 7
  cfet     drive functions, per-step weights, Lanczos recurrence, small
           tridiagonal exponential, CFET step loop, dense (expm) mode

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
facts the paper or mathematics fixes (printed values, closed forms, library
routines on special cases, convergence orders, invariants).
"""
from . import schemes, cfet  # noqa: F401
