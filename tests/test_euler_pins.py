"""Pins of the oracle's two-dimensional incompressible flow and its strategy-1
means (pseudospectral and semi-Lagrangian, appendix B): exact steady and
uniform flows, conservation of energy and enstrophy, and material conservation
of vorticity (eq. (4.2)) with the error ordering the paper reports."""

import math

import numpy as np
import pytest

from oracle.euler2d import Euler2D
from synth.euler import two_vortex_vorticity
from test_oracle_pins import _grid


def _run(N, dt, zeta0, steps, **kw):
    e = Euler2D(N, dt, zeta0, **kw)
    e.begin_interval()
    e.step(steps)
    return e, e.end_interval()


@pytest.mark.parametrize("interp", ["bilinear", "cubic"])
def test_steady_shear_flow_is_exact_for_both_discretisations(interp):
    # zeta = A cos(y) + B sin(2y): u = u(y), v = 0, u . grad zeta = 0, steady;
    # particles move along x, so zeta~ = zeta and eta_x = u T / 2, eta_y = 0
    N, dt, steps = 32, 0.01, 60
    X, Y = _grid(N)
    A, B = 0.7, -0.4
    zeta = A * np.cos(Y) + B * np.sin(2 * Y)
    u = -A * np.sin(Y) + 0.5 * B * np.cos(2 * Y)     # -dpsi/dy with lap psi = zeta
    e, out = _run(N, dt, zeta, steps, interp=interp)
    T = steps * dt
    assert np.max(np.abs(out["zeta"] - zeta)) < 1e-13
    for k in ("PS_mean", "SL_mean"):
        assert np.max(np.abs(out[k] - zeta)) < 1e-12, k
    for k in ("PS_eta_x", "SL_eta_x"):
        assert np.max(np.abs(out[k] - u * T / 2)) < 1e-12, k
    for k in ("PS_eta_y", "SL_eta_y"):
        assert np.max(np.abs(out[k])) < 1e-13, k


def test_uniform_flow_gives_half_the_displacement():
    # no vorticity, uniform (U0, V0): x - Xi^{-1} = U T / 2 in both discretisations
    N, dt, steps = 16, 0.02, 37
    U0, V0 = 0.3, -0.55
    e, out = _run(N, dt, np.zeros((N, N)), steps, U0=U0, V0=V0)
    T = steps * dt
    for k in ("PS", "SL"):
        assert np.max(np.abs(out[f"{k}_eta_x"] - U0 * T / 2)) < 1e-13
        assert np.max(np.abs(out[f"{k}_eta_y"] - V0 * T / 2)) < 1e-13
        assert np.max(np.abs(out[f"{k}_mean"])) < 1e-14


def test_energy_and_enstrophy_are_conserved():
    N, dt = 64, 0.005
    e = Euler2D(N, dt, two_vortex_vorticity(N))
    k2 = e.G.KX ** 2 + e.G.KY ** 2
    w = np.where(e.G.KX == 0, 1.0, 2.0)   # rfft2 half-plane weights

    def invariants():
        z = e.Y["zeta"]
        return np.sum(w * np.abs(z) ** 2 * e.inv_k2), np.sum(w * np.abs(z) ** 2)
    E0, Z0 = invariants()
    e.step(400)
    E1, Z1 = invariants()
    assert abs(E1 - E0) / E0 < 1e-6 and abs(Z1 - Z0) / Z0 < 1e-4


def test_material_conservation_of_vorticity_with_the_papers_ordering():
    # zeta~^L(x, tau) = zeta(x, tau + T) (eq. (4.2)): pseudospectral best,
    # semi-Lagrangian cubic better than linear (the paper's figure 2), and the
    # semi-Lagrangian errors converge with N
    T_steps, dt = 400, 0.005
    err = {}
    for N in (32, 64):
        for interp in ("bilinear", "cubic"):
            _, out = _run(N, dt, two_vortex_vorticity(N), T_steps, interp=interp)
            ref = out["zeta"]
            nrm = np.linalg.norm(ref)
            err[(N, interp)] = np.linalg.norm(out["SL_mean"] - ref) / nrm
            err[(N, "ps")] = np.linalg.norm(out["PS_mean"] - ref) / nrm
    for N in (32, 64):
        assert err[(N, "ps")] < err[(N, "cubic")] < err[(N, "bilinear")], err
    assert err[(64, "ps")] < 1e-5, err
    # linear interpolation at small Courant number c = u dt / dx acts as a
    # diffusion of about u dx / 2: first order in dx; cubic is much higher order
    # until the first-order departure point Y = X - dt u(X) limits it
    assert err[(32, "bilinear")] / err[(64, "bilinear")] > 1.7, err
    assert err[(32, "cubic")] / err[(64, "cubic")] > 3.0, err
