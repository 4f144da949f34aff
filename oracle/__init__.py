"""Plain FP64 CPU oracle of the SWR-Galerkin method (Lorin, arXiv 1710.02401).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package: only the test suite, the smoke check of the
graft entry point and the CPU-baseline leg of the benchmark use it.  It
shares no code with the HIP library (no kernels, headers, tables or
helpers); both read their inputs from the `workloads` package, which holds
parameters and seeded draws only.

Every routine follows the paper's definitions in the paper's order, with
library primitives (NumPy/SciPy: erf, Gauss-Legendre rule, dense solve,
symmetric eigensolver) as single steps and no blocking, fusion or
reordering beyond what those definitions state.

Where the paper is silent or garbled the oracle takes the readings listed
in the design notes; each module names the passage it follows.

Pinning status (what checks each part against something other than
itself) is given per module; all parts are pinned by tests under `tests/`
(closed forms, textbook special cases, invariants, brute force) except
where a module header says "parity unpinned".
"""
from . import gauss1d, geometry, quadrature, lsd, lo2, slater, assemble, swr, tise, reconstruct, mlp, learned  # noqa: F401
