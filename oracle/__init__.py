"""FP64 CPU oracle of the multirate MRT lattice-Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP path: the only
common module is ``lbm_inputs`` (seeded parameter sets, no arithmetic of the
method).

The oracle is deliberately plain: whole-grid NumPy passes in float64, the
literal moment-space collision of Eq. (14) with the transformation matrices
as printed (Eq. 16) or stated for the reduced lattices, explicit streaming with
boundary masks, and the multirate loop of Eq. (34) with the phase-step
transfer of Eq. (36)-(39).  Every function cites the passage it follows.

Parity pins: every routine is checked by ``tests/test_oracle_*.py`` against
closed forms, invariants, printed numbers and brute-force loops: the
inlet/outflow columns by an empty channel's fixed point and inlet-flux
balance, the accumulated coupling by its conservation invariant and the
order of its injection, the 3D extension by its own closed forms and
symmetries.  Long-run tip velocities, which the paper prints only as curves
against data that is not available, remain parity unpinned.
"""

from . import lattice, params, stencils, model, diag  # noqa: F401
from .model import Domain, run  # noqa: F401
