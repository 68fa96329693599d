"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package builds initial conditions (turbulent geostrophic flow plus a band of
Poincare waves) and the workload table.  It holds none of the Lagrangian-mean
arithmetic and none of the shallow-water time stepping: it only draws random
phases and assembles plane waves whose polarisation follows linear
shallow-water theory (the mode-1 wave of the paper's section 4.2.1 generalised
to an arbitrary wavevector).
"""

from .fields import turbulence_plus_waves, geostrophic_field, wave_field, linear_energy
from .workloads import Workload, WORKLOADS, workload, nu8_rule, averaging_steps

__all__ = [
    "turbulence_plus_waves",
    "geostrophic_field",
    "wave_field",
    "linear_energy",
    "Workload",
    "WORKLOADS",
    "workload",
    "nu8_rule",
    "averaging_steps",
]
