"""Plain, slow FP64 CPU oracle of ChASE (Chebyshev Accelerated Subspace iteration Eigensolver).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the HIP library under ``paper_1805_10121_amd/`` and imports nothing from
it.  Inputs come from the seeded generators (a module that holds none of the method's
arithmetic) or from the tests themselves.

Everything is NumPy complex128 / float64.  Library primitives used as single steps: ``@``
(matmul), ``numpy.linalg.qr`` (Householder QR), ``numpy.linalg.eigh`` (dense Hermitian
eigensolver, playing the role of TSOLVE), ``numpy.linalg.norm``.

Modules
-------
chebyshev : Def. 4.1 / Eq. (2)-(5) closed forms, Alg. 4 / Eq. (7) filter (two transcriptions).
lanczos   : Alg. 6 (k-step Lanczos, upper bound b_sup, DoS estimate of mu_1 and mu_{nev+nex}).
chase     : Alg. 1 driver with Alg. 2 (Rayleigh-Ritz), Alg. 3 (deflation & locking),
            Alg. 5 (degrees), plus the sequence driver (warm start, Sec. 3.3).

Parity status per function is stated in each module header.  Every function has a pin; for
the DoS estimate of mu_{nev+nex} (``lanczos.dos_estimates``) the pins are the cases the
mathematics fixes (Gauss quadrature, the counting function at full length), while how well a
few short runs estimate a large spectrum remains a heuristic.
"""

from . import chebyshev, lanczos, chase  # noqa: F401
from .chase import ChaseParams, solve, solve_sequence  # noqa: F401
from .chebyshev import filter_columns, filter_alg4, filter_scalars  # noqa: F401
