"""CPU reference ("oracle") for the entanglement-aware MPS/MPO gate update.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library; the only thing both sides read is the seeded input generator module
``circuits``.

Everything here is plain, slow and complex128:

* :mod:`oracle.jacobi`  -- one-sided (Hestenes) Jacobi SVD written out.
* :mod:`oracle.mps`     -- MPS (pure, d=2) / MPO (mixed, d=4) simulator with a
  single orthogonality centre, the two-site update, the truncation rule, the
  running fidelity estimate and the target schedules (paper Secs. II-VI,
  Eqs. (2), (4)-(6), (10)-(14)).
* :mod:`oracle.brute`   -- brute-force state-vector / density-matrix
  simulators and the fidelities of Eqs. (7) and (9).
* :mod:`oracle.adjoint` -- FP64 reverse-mode gradient of an energy through
  the updates with kept ranks frozen.
* :mod:`oracle.vidal`   -- the layer-parallel gauge (Vidal form, Hastings'
  update): all disjoint gates of a layer from the estimate before it.
* :mod:`oracle.topk`    -- the partial (top-k) factorisation: randomized
  subspace iteration from a SplitMix64 start block, the kept rank from the
  Ritz values plus the weight outside the subspace.

Parity status: every function is pinned by a ``-m "not gpu"`` test against
brute force, a closed form, an invariant or a library routine, except the
multi-truncation product estimate of Eq. (12), which the paper only states
as an approximation ("parity unpinned": checked softly, never asserted).
"""
from .jacobi import jacobi_svd, JacobiResult  # noqa: F401
from .mps import OracleMPS, truncation_rule  # noqa: F401
from . import brute  # noqa: F401
