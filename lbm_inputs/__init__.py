"""Seeded synthetic workloads for the multirate lattice-Boltzmann hot path.

This module is shared by the FP64 oracle and the HIP path.  It holds only
parameter values (the numbers printed in the paper's Sections 4.1-4.4 and
Table 1, plus seeded random draws) and seed geometry.  It holds none of the
method's arithmetic: relaxation times, effective coefficients, equilibria and
every per-site quantity are computed independently by each consumer.
"""

from .configs import (  # noqa: F401
    WORKLOADS,
    workload,
    thermal_128,
    solutal_512,
    thermosolutal_flow_1024,
    thermosolutal_flow_4096,
    ensemble_256,
    directional_3d,
    directional_2d,
    thermal_forced_512,
    solutal_forced_1000,
    thermosolutal_forced_1500,
    reduced,
)
