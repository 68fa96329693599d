"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: closed forms
(exact plane-wave means, small-amplitude Stokes corrections, exact nonlinear
steady states and inertial oscillations, linear dispersion and decay), brute-force
particle tracking (the definition of the means), and invariants (mass,
potential-vorticity material conservation, strategy-1/strategy-2 consistency).
"""

import math

import numpy as np
import pytest

from oracle.closed import (adler_frequency, omega_nondimensional, omega_poincare,
                           plane_wave_exact_means, stokes_corrections)
from oracle.lagmean import Params, PlaneWave, Run, bilinear_periodic, relative_l2
from oracle.tracker import means_by_tracking


def _grid(N):
    x = np.arange(N) * 2 * np.pi / N
    return np.broadcast_to(x[None, :], (N, N)).copy(), np.broadcast_to(x[:, None], (N, N)).copy()


def _trig_interp(F, px, py):
    """Exact trigonometric interpolant of the periodic grid field F at points (px, py)."""
    N = F.shape[0]
    Fh = np.fft.fft2(F) / (N * N)
    k = np.fft.fftfreq(N, d=1.0 / N)
    # drop the Nyquist row/column so the interpolant is real and unique
    keep = np.abs(k) < N / 2
    kx = k[keep]
    ky = k[keep]
    Fh = Fh[np.ix_(keep, keep)]
    ex = np.exp(1j * np.multiply.outer(px.ravel(), kx))  # (P, nkx)
    ey = np.exp(1j * np.multiply.outer(py.ravel(), ky))  # (P, nky)
    val = np.einsum("pj,jk,pk->p", ey, Fh, ex)
    return np.real(val).reshape(px.shape)


# ---------------------------------------------------------------- printed values

def test_dispersion_reproduces_printed_frequency():
    # section 4.2.1: Ro = 0.1, Fr = 0.5 give omega = 10.2
    assert abs(omega_nondimensional(0.1, 0.5) - 10.2) < 5e-3


def test_printed_interval_is_about_3p6_wave_periods():
    # section 4.2.1: T = 2.2 corresponds to about 3.6 wave periods
    om = omega_nondimensional(0.1, 0.5)
    assert abs(2.2 * om / (2 * math.pi) - 3.6) < 0.05


# ---------------------------------------------------------------- helpers of the oracle

def test_bilinear_exact_for_whole_and_half_cell_shifts_and_linear_data():
    N = 16
    dx = 2 * np.pi / N
    rng = np.random.default_rng(0)
    F = rng.standard_normal((N, N))
    X, Y = _grid(N)
    # whole-cell shift: +2 cells in x, -3 in y -> exact sample of the shifted grid
    G = bilinear_periodic(F, np.full((N, N), 2 * dx), np.full((N, N), -3 * dx), dx)
    assert np.array_equal(G, np.roll(np.roll(F, -2, axis=1), 3, axis=0))
    # half-cell shift in x: average of the two neighbours
    G = bilinear_periodic(F, np.full((N, N), 0.5 * dx), np.zeros((N, N)), dx)
    assert np.allclose(G, 0.5 * (F + np.roll(F, -1, axis=1)), atol=1e-15)
    # bilinear data away from the periodic seam is reproduced exactly
    L = 3.0 + 0.7 * X - 0.2 * Y + 0.05 * X * Y
    ox = 0.37 * dx
    oy = -0.81 * dx
    G = bilinear_periodic(L, np.full((N, N), ox), np.full((N, N), oy), dx)
    inner = (slice(2, N - 2), slice(2, N - 2))
    exact = 3.0 + 0.7 * (X + ox) - 0.2 * (Y + oy) + 0.05 * (X + ox) * (Y + oy)
    assert np.allclose(G[inner], exact[inner], atol=1e-13)


def test_vorticity_sign_and_derivatives_in_dynamic_mode():
    # zeta = dv/dx - du/dy: for u = -sin y, v = sin x it is cos x + cos y.  The
    # Eulerian mean over one tiny step returns zeta at the start.
    N = 32
    X, Y = _grid(N)
    u, v, h = -np.sin(Y), np.sin(X), np.ones((N, N))
    r = Run(Params(N=N, dt=1e-7, fields=("zeta",)), u, v, h)
    r.begin_interval()
    r.step(1)
    out = r.end_interval()
    assert np.max(np.abs(out["E_mean:zeta"] - (np.cos(X) + np.cos(Y)))) < 1e-6


# ---------------------------------------------------------------- dynamics

def test_mass_is_conserved_to_roundoff():
    from synth import workload
    w = workload("sw64_fp64")
    u, v, h = w.initial_state()
    r = Run(Params(N=64, dt=w.dt, nu8=w.nu8), u, v, h)
    m0 = r.Y["h"][0, 0].real
    r.begin_interval()
    r.step(30)
    out = r.end_interval()
    assert abs(r.Y["h"][0, 0].real - m0) / abs(m0) < 1e-14
    # the domain mean of the Eulerian mean depth is the (conserved) mean depth
    assert abs(out["E_mean:h"].mean() - 1.0) < 1e-13


def test_inertial_oscillation_is_exact_and_means_of_uniform_fields():
    # uniform (u, v) with flat h is an exact nonlinear solution: an inertial
    # oscillation u + i v = (U + i V) exp(-i f t).  No Stokes drift: L = E for u.
    N = 16
    U, V, f = 0.3, -0.1, 1.0
    dt = 0.01
    n = 200
    r = Run(Params(N=N, dt=dt, f=f, fields=("h", "u", "v")),
            np.full((N, N), U), np.full((N, N), V), np.ones((N, N)))
    r.begin_interval()
    r.step(n)
    out = r.end_interval()
    t = n * dt
    uu, vv, hh = r.dynamics_physical()
    ue = U * math.cos(f * t) + V * math.sin(f * t)
    ve = V * math.cos(f * t) - U * math.sin(f * t)
    assert np.max(np.abs(uu - ue)) < 1e-9 and np.max(np.abs(vv - ve)) < 1e-9
    assert np.max(np.abs(hh - 1.0)) < 1e-14
    for key in ("S1_mean:h", "S2_mean:h", "E_mean:h"):
        assert np.max(np.abs(out[key] - 1.0)) < 1e-13
    for comp in ("u", "v"):
        for S in ("S1", "S2"):
            assert np.max(np.abs(out[f"{S}_mean:{comp}"] - out[f"E_mean:{comp}"])) < 1e-12
    # displacements are uniform
    for key in ("S2_xi_x", "S2_xi_y", "S1_eta_x", "S1_eta_y"):
        assert np.ptp(out[key]) < 1e-13


@pytest.mark.parametrize("axis", ["x", "y"])
def test_geostrophic_jet_is_an_exact_steady_state(axis):
    # u = U sin y, h = H + (f U / g) cos y (and its rotated twin) is steady for the
    # full nonlinear equations: pins the zeta u / zeta v and kinetic-energy terms.
    N = 32
    X, Y = _grid(N)
    U, f, g = 0.2, 1.0, 1.0
    if axis == "x":
        u, v, h = U * np.sin(Y), np.zeros((N, N)), 1.0 + (f * U / g) * np.cos(Y)
    else:
        u, v, h = np.zeros((N, N)), U * np.sin(X), 1.0 - (f * U / g) * np.cos(X)
    r = Run(Params(N=N, dt=0.05), u, v, h)
    r.step(40)
    uu, vv, hh = r.dynamics_physical()
    assert np.max(np.abs(uu - u)) < 1e-13
    assert np.max(np.abs(vv - v)) < 1e-13
    assert np.max(np.abs(hh - h)) < 1e-13


@pytest.mark.parametrize("kvec", [(2, 0), (5, 3)])
def test_linear_wave_propagates_with_poincare_frequency_and_hyperviscous_decay(kvec):
    # small-amplitude plane wave: the field at time t is the linear solution
    # (frequency sqrt(f^2 + g H |k|^2), decay exp(-nu8 |k|^8 t)) up to O(A^2)
    N = 32
    X, Y = _grid(N)
    kx, ky = kvec
    k2 = kx * kx + ky * ky
    om = omega_poincare(math.sqrt(k2))
    nu8 = 1e-7   # dt nu8 |k|^8 stays inside RK4's stability region up to the mask corner
    A = 1e-6

    def wave(t):
        th = kx * X + ky * Y - om * t
        c, s = np.cos(th), np.sin(th)
        d = math.exp(-nu8 * k2 ** 4 * t)
        return (d * A * (om * kx * c - ky * s) / k2, d * A * (om * ky * c + kx * s) / k2,
                1.0 + d * A * c)

    u, v, h = wave(0.0)
    dt = 0.01
    n = 150
    r = Run(Params(N=N, dt=dt, nu8=nu8), u, v, h)
    r.step(n)
    uu, vv, hh = r.dynamics_physical()
    ue, ve, he = wave(n * dt)
    for a, b in ((uu, ue), (vv, ve), (hh - 1.0, he - 1.0)):
        assert np.max(np.abs(a - b)) < 1e-3 * A


def test_energy_is_nearly_conserved_without_dissipation():
    # inviscid shallow water conserves E = 1/2 <h |u|^2 + g h^2>; the truncated
    # system drifts only slightly over a smooth, well-resolved evolution
    from synth import turbulence_plus_waves
    N = 32
    u, v, h = turbulence_plus_waves(N, k0=2.0, Ro=0.05, k_lo=1.0, k_hi=2.0, ratio=0.5,
                                    seed_vortex=11, seed_wave=12)
    r = Run(Params(N=N, dt=0.01, nu8=0.0), u, v, h)

    def energy():
        uu, vv, hh = r.dynamics_physical()
        return 0.5 * np.mean(hh * (uu * uu + vv * vv) + hh * hh)

    e0 = energy()
    r.step(200)
    e1 = energy()
    ek = 0.5 * np.mean(u * u + v * v)
    assert abs(e1 - e0) < 1e-4 * ek


# ---------------------------------------------------------------- Lagrangian means: closed forms

def _plane_wave_run(N, k=2.0, a=0.3, m=1, nsteps=400, fields=("h", "u", "v")):
    omega = omega_poincare(k)
    A = k * a / omega
    Om = adler_frequency(k, a, omega)
    dt = m * 2 * math.pi / Om / nsteps
    p = Params(N=N, dt=dt, fields=fields, mode="kinematic", waves=[PlaneWave(k, 0.0, A, omega)])
    r = Run(p)
    r.begin_interval()
    r.step(nsteps)
    return r.end_interval(), plane_wave_exact_means(k, a, omega), (k, a, omega, nsteps * dt)


def test_plane_wave_exact_means_both_strategies():
    # Adler-equation solution: every particle has the same mean velocity and depth
    errs = {}
    outs = {}
    for N in (32, 64):
        out, (uL, vL, hL), wave = _plane_wave_run(N)
        outs[N] = out
        for key, ex in (("u", uL), ("v", vL), ("h", hL)):
            errs[(N, "S1", key)] = np.max(np.abs(out[f"S1_mean:{key}"] - ex))
            errs[(N, "S2", key)] = np.max(np.abs(out[f"S2_mean:{key}"] - ex))
    for key in ("u", "v", "h"):
        assert errs[(64, "S1", key)] < 1e-7          # spectral in space, RK4 in time
        assert errs[(64, "S2", key)] < 5e-4          # bilinear interpolation, O(dx^2)
        assert errs[(32, "S2", key)] / errs[(64, "S2", key)] > 3.0
    # the Eulerian mean is the plain time average at fixed x:
    # (1/T) int a cos(k x - omega t) dt = a (sin(k x) - sin(k x - omega T)) / (omega T)
    k, a, omega, T = wave
    X, _ = _grid(32)
    e_exact = a * (np.sin(k * X) - np.sin(k * X - omega * T)) / (omega * T)
    assert np.max(np.abs(outs[32]["E_mean:u"] - e_exact)) < 1e-9
    assert uL > 0.02    # the Lagrangian mean velocity is a genuine drift


def test_uniform_flow_displacements_are_exact():
    # steady uniform flow: partial mean position moves at U/2, so xi = U s / 2 and
    # P = U s^2 / 2, i.e. eta = x - Xi^{-1} = U T / 2; every mean equals the field
    N = 16
    U, V = 0.4, -0.25
    dt = 0.03
    p = Params(N=N, dt=dt, fields=("h", "u", "one"), mode="kinematic", U0=U, V0=V)
    r = Run(p)
    r.step(5)
    for _ in range(2):   # two consecutive intervals give identical results
        r.begin_interval()
        r.step(37)
        out = r.end_interval()
        T = 37 * dt
        assert np.max(np.abs(out["S2_xi_x"] - U * T / 2)) < 1e-14
        assert np.max(np.abs(out["S2_xi_y"] - V * T / 2)) < 1e-14
        assert np.max(np.abs(out["S1_eta_x"] - U * T / 2)) < 1e-14
        assert np.max(np.abs(out["S1_eta_y"] - V * T / 2)) < 1e-14
        for S in ("S1", "S2", "E"):
            assert np.max(np.abs(out[f"{S}_mean:h"] - 1.0)) < 1e-14
            assert np.max(np.abs(out[f"{S}_mean:u"] - U)) < 1e-14
            assert np.max(np.abs(out[f"{S}_mean:one"] - 1.0)) < 1e-14


def test_rest_state_gives_zero_displacement_and_identity_means():
    N = 16
    r = Run(Params(N=N, dt=0.05), np.zeros((N, N)), np.zeros((N, N)), np.ones((N, N)))
    r.begin_interval()
    r.step(10)
    out = r.end_interval()
    for key in ("S2_xi_x", "S2_xi_y", "S1_eta_x", "S1_eta_y", "S1_mean:zeta", "S2_mean:zeta"):
        assert np.max(np.abs(out[key])) < 1e-15
    for key in ("S1_mean:h", "S2_mean:h", "E_mean:h"):
        assert np.max(np.abs(out[key] - 1.0)) < 1e-15


def test_stokes_corrections_of_a_small_amplitude_wave_in_the_full_dynamics():
    # Lagrangian minus Eulerian means of a weak Poincare wave averaged over two
    # periods: u_S = k a^2/(2 omega), h: H k^2 a^2/(2 omega^2), v: 0
    N = 32
    k = 2.0
    om = omega_poincare(k)
    X, _ = _grid(N)
    devs = {}
    for a in (0.02, 0.01):
        u, v, h = a * np.cos(k * X), (a / om) * np.sin(k * X), 1.0 + (k * a / om) * np.cos(k * X)
        nsteps = 400
        r = Run(Params(N=N, dt=2 * 2 * math.pi / om / nsteps, fields=("h", "u", "v")), u, v, h)
        r.begin_interval()
        r.step(nsteps)
        out = r.end_interval()
        du, dv, dh = stokes_corrections(k, a, om)
        for key, th in (("u", du), ("h", dh)):
            for S in ("S1", "S2"):
                d = (out[f"{S}_mean:{key}"] - out[f"E_mean:{key}"]).mean()
                devs[(a, S, key)] = abs(d - th) / th
        for S in ("S1", "S2"):
            dvm = (out[f"{S}_mean:v"] - out[f"E_mean:v"]).mean()
            assert abs(dvm) < 0.01 * du
    for key in ("u", "h"):
        assert devs[(0.02, "S1", key)] < 1e-3
        # S1 deviation is O(a^2) relative: halving a divides it by about 4
        assert devs[(0.02, "S1", key)] / devs[(0.01, "S1", key)] > 3.0
        # S2 carries the bilinear O((k dx)^2) relative error on top
        assert devs[(0.02, "S2", key)] < 0.025


# ---------------------------------------------------------------- Lagrangian means: definition

TWO_WAVES = [PlaneWave(1.0, 1.0, 0.08, math.sqrt(3.0), 0.3),
             PlaneWave(2.0, -1.0, 0.05, math.sqrt(6.0), 1.1)]


def _tracked_case(N, nsteps=200, dt=0.02, n_tau=3):
    p = Params(N=N, dt=dt, fields=("h", "u"), mode="kinematic", waves=TWO_WAVES,
               U0=0.05, V0=-0.03)
    r = Run(p)
    r.step(n_tau)
    r.begin_interval()
    r.step(nsteps)
    out = r.end_interval()
    tr = means_by_tracking(p, n_tau, nsteps, ("h", "u"))
    return out, tr


def test_means_converge_to_brute_force_particle_tracking():
    err = {}
    for N in (16, 32):
        out, tr = _tracked_case(N)
        for key in tr:
            err[(N, key)] = np.max(np.abs(out[key] - tr[key]))
    # strategy 1 is spectral in space: fast convergence to the tracked means
    for key in ("S1_mean:h", "S1_mean:u", "S1_eta_x", "S1_eta_y"):
        assert err[(32, key)] < 1e-7
        assert err[(16, key)] / err[(32, key)] > 100.0
    # strategy 2 uses bilinear interpolation: second order
    for key in ("S2_mean:h", "S2_mean:u", "S2_xi_x", "S2_xi_y"):
        assert err[(32, key)] < 2e-3
        assert err[(16, key)] / err[(32, key)] > 2.8


def test_strategy1_and_strategy2_describe_the_same_particles():
    # f~^L(x + xi(x)) = f-bar^L(x) and eta(x + xi(x)) = xi(x): both strategies give
    # "end position minus mean position" and the mean along one trajectory
    N = 32
    out, _ = _tracked_case(N)
    X, Y = _grid(N)
    px = X + out["S2_xi_x"]
    py = Y + out["S2_xi_y"]
    for s1, s2 in (("S1_mean:h", "S2_mean:h"), ("S1_mean:u", "S2_mean:u"),
                   ("S1_eta_x", "S2_xi_x"), ("S1_eta_y", "S2_xi_y")):
        interp = _trig_interp(out[s1], px, py)
        assert np.max(np.abs(interp - out[s2])) < 2e-3
        # and the error is the S2 discretisation error, not a mismatch of meaning
        assert np.max(np.abs(interp - out[s2])) < 0.2 * np.max(np.abs(out[s2] - out[s2].mean()))


def _smooth_flow(N):
    """The same smooth balanced flow plus a Poincare wave at every N (analytic)."""
    X, Y = _grid(N)
    a1, a2 = 0.05, 0.03
    psi = a1 * np.sin(X) * np.cos(Y) + a2 * np.cos(2 * X - Y + 0.4)
    u = a1 * np.sin(X) * np.sin(Y) + a2 * (-np.sin(2 * X - Y + 0.4))
    v = a1 * np.cos(X) * np.cos(Y) + a2 * (-2 * np.sin(2 * X - Y + 0.4))
    A, kx, ky = 0.02, 1.0, 1.0
    om = omega_poincare(math.sqrt(2.0))
    th = kx * X + ky * Y + 0.7
    u = u + A * (om * kx * np.cos(th) - ky * np.sin(th)) / 2.0
    v = v + A * (om * ky * np.cos(th) + kx * np.sin(th)) / 2.0
    h = 1.0 + psi + A * np.cos(th)
    return u, v, h


def test_potential_vorticity_means_follow_material_conservation():
    # q = (f + zeta)/h is materially conserved without dissipation: strategy 1
    # gives q~^L(x) = q(x, tau+T) and strategy 2 gives q-bar^L(x) = q(x + xi(x), tau+T)
    res = {}
    for N in (32, 64):
        u, v, h = _smooth_flow(N)
        r = Run(Params(N=N, dt=0.02, nu8=0.0, fields=("q",)), u, v, h)
        r.begin_interval()
        r.step(100)
        out = r.end_interval()
        uu, vv, hh = r.dynamics_physical()
        zz = np.fft.irfft2(1j * r.grid.KX * r.Y["v"] - 1j * r.grid.KY * r.Y["u"], s=(N, N))
        q = (1.0 + zz) / hh
        X, Y = _grid(N)
        res[(N, "S1")] = relative_l2(out["S1_mean:q"] - 1.0, q - 1.0)
        q_at = _trig_interp(q, X + out["S2_xi_x"], Y + out["S2_xi_y"])
        res[(N, "S2")] = relative_l2(out["S2_mean:q"] - 1.0, q_at - 1.0)
    assert res[(64, "S1")] < 1e-9
    assert res[(32, "S1")] / res[(64, "S1")] > 1e3     # spectral convergence
    assert res[(64, "S2")] < 3e-3
    # bilinear gathers: the interpolation error has kinks where xi/dx crosses an
    # integer, so its gradient (advected by w) is O(dx) and the order drops below 2
    assert res[(32, "S2")] / res[(64, "S2")] > 2.0


def test_averaging_is_linear_and_exact_for_constants():
    from synth import turbulence_plus_waves
    N = 32
    u, v, h = turbulence_plus_waves(N, k0=2.0, Ro=0.05, k_lo=1.0, k_hi=2.0, ratio=1.0,
                                    seed_vortex=5, seed_wave=6)
    r = Run(Params(N=N, dt=0.02, fields=("one", "u", "v", "h")), u, v, h)
    r.begin_interval()
    r.step(20)
    out = r.end_interval()
    for S in ("S1", "S2", "E"):
        assert np.max(np.abs(out[f"{S}_mean:one"] - 1.0)) < 1e-13
    # each averaged field evolves on its own: the means of h do not depend on
    # which other fields are averaged alongside
    r2 = Run(Params(N=N, dt=0.02, fields=("h",)), u, v, h)
    r2.begin_interval()
    r2.step(20)
    out2 = r2.end_interval()
    for S in ("S1", "S2", "E"):
        assert np.max(np.abs(out2[f"{S}_mean:h"] - out[f"{S}_mean:h"])) < 1e-14
