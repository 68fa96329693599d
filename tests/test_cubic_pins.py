"""Pins of the oracle's cubic gather (the strategy-2 interpolation option):
exact shifts, exactness for cubic polynomials, fourth-order convergence, and
the plane-wave means of strategy 2 against their closed form."""

import math

import numpy as np

from oracle.closed import adler_frequency, omega_poincare, plane_wave_exact_means
from oracle.lagmean import Params, PlaneWave, Run, cubic_periodic
from test_oracle_pins import _grid


def test_zero_and_whole_cell_offsets_are_exact():
    N = 16
    dx = 2 * np.pi / N
    rng = np.random.default_rng(5)
    F = rng.standard_normal((N, N))
    z = np.zeros((N, N))
    assert np.array_equal(cubic_periodic(F, z, z, dx), F)
    got = cubic_periodic(F, np.full((N, N), -2 * dx), np.full((N, N), 5 * dx), dx)
    assert np.max(np.abs(got - np.roll(np.roll(F, 2, axis=1), -5, axis=0))) < 1e-14


def test_cubic_polynomials_are_reproduced():
    # F = a bicubic polynomial of the grid indices; query points whose 4 x 4
    # stencil does not wrap get the polynomial's value exactly
    N = 32
    dx = 2 * np.pi / N
    rng = np.random.default_rng(6)
    C = rng.standard_normal((4, 4))
    P = lambda x, y: sum(C[j, i] * (x / N) ** i * (y / N) ** j for i in range(4) for j in range(4))
    I = np.arange(N, dtype=np.float64)
    F = P(I[None, :], I[:, None])
    ox = rng.uniform(-1.5, 1.5, (N, N))
    oy = rng.uniform(-1.5, 1.5, (N, N))
    got = cubic_periodic(F, ox * dx, oy * dx, dx)
    want = P(I[None, :] + ox, I[:, None] + oy)
    inner = np.zeros((N, N), dtype=bool)
    inner[4:N - 4, 4:N - 4] = True
    assert np.max(np.abs(got - want)[inner]) < 1e-12


def test_fourth_order_on_a_smooth_field():
    errs = []
    for N in (16, 32, 64):
        X, Y = _grid(N)
        dx = 2 * np.pi / N
        rng = np.random.default_rng(7)
        ox = rng.uniform(-2, 2, (N, N)) * dx
        oy = rng.uniform(-2, 2, (N, N)) * dx
        f = lambda x, y: np.sin(x + 0.3) * np.cos(2 * y) + 0.5 * np.cos(x - y)
        errs.append(np.max(np.abs(cubic_periodic(f(X, Y), ox, oy, dx) - f(X + ox, Y + oy))))
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 13, errs


def _plane_wave_s2(N, interp, k=2.0, a=0.3, nsteps=400):
    omega = omega_poincare(k)
    A = k * a / omega
    dt = 2 * math.pi / adler_frequency(k, a, omega) / nsteps
    p = Params(N=N, dt=dt, fields=("h", "u", "v"), mode="kinematic", waves=[PlaneWave(k, 0.0, A, omega)],
               interp=interp)
    r = Run(p)
    r.begin_interval()
    r.step(nsteps)
    out = r.end_interval()
    uL, vL, hL = plane_wave_exact_means(k, a, omega)
    return max(np.max(np.abs(out[f"S2_mean:{key}"] - ex)) for key, ex in (("u", uL), ("v", vL), ("h", hL)))


def test_strategy2_plane_wave_means_with_cubic_gathers():
    e_lin = {N: _plane_wave_s2(N, "bilinear") for N in (32, 64)}
    e_cub = {N: _plane_wave_s2(N, "cubic") for N in (32, 64)}
    assert e_cub[32] < e_lin[32] / 10 and e_cub[64] < e_lin[64] / 10, (e_lin, e_cub)
    assert e_cub[32] / e_cub[64] > 8, e_cub
