"""Closed forms used to pin the oracle.

TEST INFRASTRUCTURE ONLY.

* Linear dispersion of Poincare waves, omega^2 = f^2 + g H |k|^2 (the paper's
  section 4.2.1 quotes omega = (Ro^-2 + Fr^-2)^(1/2) = 10.2 for Ro = 0.1, Fr = 0.5,
  which is this relation in its non-dimensional form with |k| = 1).
* Exact means for a prescribed plane wave.  For u = a cos(theta),
  v = (f a / omega) sin(theta), h = H + (H k a / omega) cos(theta),
  theta = k x - omega t, the particle phase psi = k phi_x - omega t obeys
  d psi/dt = k a cos(psi) - omega, an Adler equation.  For omega > k a its
  period is 2 pi / Omega with Omega = sqrt(omega^2 - k^2 a^2), during which the
  particle moves by 2 pi (omega - Omega) / (k Omega).  Averaged over a whole
  number of such periods, every particle therefore has
      mean u = u_L = (omega - Omega) / k,   mean v = 0,
      mean h = H + H k u_L / omega,
  and these are both the strategy-1 and strategy-2 means (they do not depend
  on the particle).  The mean of cos(psi) in time is (omega - Omega)/(k a).
* Small-amplitude limit of the same wave in the full dynamics: Lagrangian minus
  Eulerian mean (Stokes correction) u_S = k a^2 / (2 omega) for u and
  H k^2 a^2 / (2 omega^2) for h, zero for v.
"""

from __future__ import annotations

import math


def omega_poincare(k: float, f: float = 1.0, g: float = 1.0, H: float = 1.0) -> float:
    return math.sqrt(f * f + g * H * k * k)


def omega_nondimensional(Ro: float, Fr: float) -> float:
    """Mode-1 frequency in the paper's non-dimensional variables (f = 1/Ro, gH = 1/Fr^2)."""
    return math.sqrt(Ro ** -2 + Fr ** -2)


def adler_frequency(k: float, a: float, omega: float) -> float:
    return math.sqrt(omega * omega - k * k * a * a)


def plane_wave_exact_means(k: float, a: float, omega: float, H: float = 1.0):
    """(u_L, v_L, h_L) for the prescribed plane wave, averaged over whole Adler periods."""
    Om = adler_frequency(k, a, omega)
    uL = (omega - Om) / k
    return uL, 0.0, H + H * k * uL / omega


def stokes_corrections(k: float, a: float, omega: float, H: float = 1.0):
    """Small-amplitude Lagrangian-minus-Eulerian means (du, dv, dh) of the plane wave."""
    return k * a * a / (2.0 * omega), 0.0, H * k * k * a * a / (2.0 * omega * omega)
