"""The seeded input generator: scaling, balance and wave polarisation."""

import math

import numpy as np

from synth import geostrophic_field, linear_energy, turbulence_plus_waves, wave_field
from synth.workloads import WORKLOADS, averaging_steps, batch_workloads, nu8_rule, serving_requests


def _ddx(a):
    N = a.shape[0]
    k = np.fft.fftfreq(N, d=1.0 / N)
    return np.real(np.fft.ifft2(1j * k[None, :] * np.fft.fft2(a)))


def _ddy(a):
    N = a.shape[0]
    k = np.fft.fftfreq(N, d=1.0 / N)
    return np.real(np.fft.ifft2(1j * k[:, None] * np.fft.fft2(a)))


def test_geostrophic_field_scaling_and_balance():
    u, v, eta = geostrophic_field(64, 6.0, 0.05, 1.0, 1.0, seed=0)
    assert abs(math.sqrt(np.mean(u * u + v * v)) - 0.05) < 1e-12
    # f z x u = -g grad eta  and  div u = 0
    assert np.max(np.abs(-v + _ddx(eta))) < 1e-12
    assert np.max(np.abs(u + _ddy(eta))) < 1e-12
    assert np.max(np.abs(_ddx(u) + _ddy(v))) < 1e-12


def test_wave_field_satisfies_linear_shallow_water():
    # each component obeys the linear equations with omega = +sqrt(f^2 + gH|k|^2):
    # checked through the linear tendency of the continuity equation d eta/dt = -H div u
    # against the time derivative of the analytic propagating field.
    N = 32
    u, v, eta = wave_field(N, 2.0, 2.0, 1.0, 1.0, 1.0, seed=3)
    # the band |k| = 2 holds the 4 waves (+-2, 0), (0, +-2), all with omega = sqrt 5
    om = math.sqrt(5.0)
    # time derivative of the propagating field is -omega * (Hilbert-rotated field):
    # equivalently, at t=0, d eta/dt = -H div u must hold exactly
    deta_dt = -(_ddx(u) + _ddy(v))
    # and d u/dt - f v = -g d eta/dx  -> du/dt = v - d eta/dx
    # check d eta/dt through the phase shift: eta(t) = Re sum c e^{i(k.x - omega t)}
    N2 = N * N
    spec = np.fft.fft2(eta)
    k = np.fft.fftfreq(N, d=1.0 / N)
    KX, KY = np.meshgrid(k, k)
    # only |k| = 2 modes are present
    assert np.all(np.abs(spec[np.abs(np.hypot(KX, KY) - 2.0) > 1e-9]) < 1e-9 * N2)
    assert np.std(deta_dt) > 0.1


def test_energy_ratio_and_mean_depth():
    u, v, h = turbulence_plus_waves(64, k0=6.0, Ro=0.05, k_lo=2.0, k_hi=4.0, ratio=2.0,
                                    seed_vortex=0, seed_wave=1)
    assert abs(np.mean(h) - 1.0) < 1e-14
    ug, vg, eg = geostrophic_field(64, 6.0, 0.05, 1.0, 1.0, seed=0)
    ew = linear_energy(u - ug, v - vg, (h - 1.0) - eg, 1.0, 1.0)
    ev = linear_energy(ug, vg, eg, 1.0, 1.0)
    assert abs(ew / ev - 2.0) < 1e-12


def test_workload_rules():
    w = WORKLOADS["sw64_fp64"]
    assert w.steps_per_interval == 1012 and abs(w.nu8 - 2.644e-10) / 2.644e-10 < 1e-3
    w = WORKLOADS["sw256_fp64"]
    assert w.steps_per_interval == 2194 and w.n_intervals == 4
    w = WORKLOADS["sw1024_fp32"]
    assert w.steps_per_interval == 4676 and abs(w.nu8 - 9.116e-19) / 9.116e-19 < 1e-3
    assert averaging_steps(2.0, 0.01) == 1012
    assert nu8_rule(64, 0.01) > 0
    runs = batch_workloads()
    assert len(runs) == 64 and {r.N for r in runs} <= {128, 192, 256, 384, 512}
    reqs = serving_requests(duration=10.0)
    assert all(reqs[i].arrival < reqs[i + 1].arrival for i in range(len(reqs) - 1))
