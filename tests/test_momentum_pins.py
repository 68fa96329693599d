"""Pins of the oracle's strategy-2 mean of the momentum 1-form (appendix C):
closed forms (uniform flow, steady geostrophic jets) and convergence to the
definition (eq. (C.1)) evaluated by particle tracking."""

import numpy as np
import pytest

from oracle.lagmean import Params, Run
from oracle.tracker import kinematic_fields, kinematic_velocity_gradient, momentum_mean_by_tracking
from test_oracle_pins import TWO_WAVES, _grid


def test_kinematic_velocity_gradient_matches_finite_differences():
    p = Params(N=8, dt=0.1, mode="kinematic", waves=TWO_WAVES, U0=0.05, V0=-0.03)
    rng = np.random.default_rng(8)
    x, y = rng.uniform(0, 6.3, 50), rng.uniform(0, 6.3, 50)
    t, h = 0.37, 1e-6
    ux, uy, vx, vy = kinematic_velocity_gradient(p, x, y, t)
    up, vp, _, _ = kinematic_fields(p, x + h, y, t)
    um, vm, _, _ = kinematic_fields(p, x - h, y, t)
    assert np.max(np.abs((up - um) / (2 * h) - ux)) < 1e-8 and np.max(np.abs((vp - vm) / (2 * h) - vx)) < 1e-8
    up, vp, _, _ = kinematic_fields(p, x, y + h, t)
    um, vm, _, _ = kinematic_fields(p, x, y - h, t)
    assert np.max(np.abs((up - um) / (2 * h) - uy)) < 1e-8 and np.max(np.abs((vp - vm) / (2 * h) - vy)) < 1e-8


def test_uniform_flow_has_its_own_momentum_as_mean():
    N, U, V, dt = 16, 0.4, -0.25, 0.03
    p = Params(N=N, dt=dt, mode="kinematic", U0=U, V0=V, momentum=True)
    r = Run(p)
    r.begin_interval()
    r.step(37)
    out = r.end_interval()
    assert np.max(np.abs(out["S2_mom_x"] - U)) < 1e-14 and np.max(np.abs(out["S2_mom_y"] - V)) < 1e-14
    tr = momentum_mean_by_tracking(p, 0, 37)
    assert np.max(np.abs(tr["S2_mom_x"] - U)) < 1e-14 and np.max(np.abs(tr["S2_mom_y"] - V)) < 1e-14


@pytest.mark.parametrize("axis", ["x", "y"])
def test_steady_geostrophic_jet_has_the_jet_as_momentum_mean(axis):
    # u = (U(y), 0): phi = a + U(a_y) t, so (1/T) int phi_s^*(u . dx) ds = (U, U U' T/2)
    # and the mean map's Jacobian has d phi-bar_x / d a_y = U' T / 2: tau-bar = (U, 0).
    # The y-component cancels only with both the (delta + grad xi) pull-back and the
    # g_j d_i w_j term right.
    N = 32
    X, Y = _grid(N)
    U, f, g = 0.2, 1.0, 1.0
    if axis == "x":
        u, v, h = U * np.sin(Y), np.zeros((N, N)), 1.0 + (f * U / g) * np.cos(Y)
    else:
        u, v, h = np.zeros((N, N)), U * np.sin(X), 1.0 - (f * U / g) * np.cos(X)
    r = Run(Params(N=N, dt=0.05, momentum=True), u, v, h)
    r.begin_interval()
    r.step(60)
    out = r.end_interval()
    assert np.max(np.abs(out["S2_mom_x"] - u)) < 1e-12
    assert np.max(np.abs(out["S2_mom_y"] - v)) < 1e-12


def test_momentum_mean_converges_to_particle_tracking():
    err = {}
    for N in (16, 32):
        p = Params(N=N, dt=0.02, fields=("h",), mode="kinematic", waves=TWO_WAVES, U0=0.05, V0=-0.03,
                   momentum=True)
        r = Run(p)
        r.step(3)
        r.begin_interval()
        r.step(200)
        out = r.end_interval()
        tr = momentum_mean_by_tracking(p, 3, 200)
        for k in ("S2_mom_x", "S2_mom_y"):
            err[(N, k)] = np.max(np.abs(out[k] - tr[k]))
    for k in ("S2_mom_x", "S2_mom_y"):
        assert err[(32, k)] < 2e-3, err
        assert err[(16, k)] / err[(32, k)] > 2.8, err     # bilinear gathers: second order
