"""Plain FP64 CPU oracle for the ensemble PCG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the tests, the package's smoke check and the CPU-baseline leg of
the benchmark do.  The oracle shares no code with the HIP path: it is written
from the paper's definitions with numpy/scipy, slowly and obviously.

Modules
-------
problem     coefficient model, nine-point assembly, right-hand side, QoI weights
pcg         per-sample Jacobi / Chebyshev PCG and the lock-step ensemble emulator
sparse_grid centre-rooted piecewise-linear hierarchy, surpluses, surrogate,
            refinement, grouping and the cost-increase ratio R
adjoint     QoI, adjoint solve and dQ/dy, plus a complex-step reference

Every function cites the passage of the paper (section / equation) or the
reading of a silent point it implements.
"""

CONVERGED = 0
MAX_ITER = 1
BREAKDOWN = 2
ZERO_RHS = 3
