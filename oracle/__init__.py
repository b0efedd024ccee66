"""Plain, slow, obviously correct CPU oracle for the tiled Cholesky path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does, and the
oracle shares no code with the HIP implementation.

* ``core``  - the C oracle (FP64 tile tasks, tiled and unblocked factor and
  solve in submission order, extended-precision checkers);
* ``dag``   - access-mode dependency inference, task lists, random
  topological orders;
* ``mixed`` - mixed-precision factor emulation, refinement, x_ref.

Each function cites the passage it follows in its own docstring.  Parity
status: every function here is pinned by tests under ``tests/``
(``test_oracle_*.py``) except the mixed-precision emulation, whose factor is
"parity unpinned" bitwise (its accumulation order is the BLAS library's);
it is pinned only by exact-integer inputs and by error bounds.
"""
from . import core, dag, mixed  # noqa: F401
