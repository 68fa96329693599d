"""Initial vorticity of the two-dimensional incompressible test flow (section
4.1, eq. (4.3)): two like-signed Gaussian vortices that later merge.  Inputs
only: no dynamics here."""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def two_vortex_vorticity(N: int) -> np.ndarray:
    """exp(-(x - pi + 0.1)^2 - (y - pi + pi/3)^2) + exp(-(x - pi - 0.1)^2 - (y - pi - pi/3)^2)
    on the grid x_i = 2 pi i / N, row-major [iy][ix]."""
    x = np.arange(N) * 2.0 * math.pi / N
    X, Y = np.meshgrid(x, x, indexing="xy")
    return (np.exp(-(X - math.pi + 0.1) ** 2 - (Y - math.pi + math.pi / 3) ** 2)
            + np.exp(-(X - math.pi - 0.1) ** 2 - (Y - math.pi - math.pi / 3) ** 2))


@dataclass(frozen=True)
class EulerWorkload:
    name: str
    N: int
    dt: float
    steps: int           # one averaging interval from tau = 0

    @property
    def T(self) -> float:
        return self.steps * self.dt

    def initial_vorticity(self) -> np.ndarray:
        return two_vortex_vorticity(self.N)


# the test of section 4.1: 128^2, dt = 0.005, T = 25
EULER_TWO_VORTEX = EulerWorkload("euler2d_two_vortex_128", 128, 0.005, 5000)
