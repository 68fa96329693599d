"""Turbulence-plus-waves initial conditions on the doubly periodic [0, 2pi)^2 grid.

Grid convention (shared by every consumer): physical arrays are N x N,
row-major [iy][ix], x_i = 2 pi i / N, float64.

Recipe (stand-in for the paper's Navier-Stokes-derived initial flow of
section 4.2.1, which is not available; all choices below are stated in the
design notes):

* geostrophic part: streamfunction with random phases, modal amplitude
  sqrt(|k|) exp(-|k|^2 / (2 k0^2)) (shell energy spectrum k^4 exp(-(k/k0)^2)),
  restricted to the dealiased square |kx|, |ky| <= floor((N-1)/3), k != 0;
  u = -d psi/dy, v = d psi/dx, eta = (f/g) psi; scaled so that the rms speed
  sqrt(<u^2 + v^2>) equals Ro * f * L with L = 1 (the first Fourier mode);
* wave part: one linear Poincare wave per integer wavevector k with
  k_lo <= |k| <= k_hi (k and -k are distinct waves), random phase, frequency
  omega = +sqrt(f^2 + g H |k|^2), equal amplitudes; the polarisation is the
  exact linear solution, which reduces to the paper's mode-1 wave for k = (1, 0);
* the wave amplitude is scaled so that the linear energy ratio
  E_wave / E_vortex equals ``ratio``, with E = 1/2 <H (u^2 + v^2) + g eta^2>.
"""

from __future__ import annotations

import numpy as np


def _int_wavenumbers(N: int):
    k = np.fft.fftfreq(N, d=1.0 / N)  # integer wavenumbers in FFT order
    KX = k[None, :].repeat(N, axis=0)
    KY = k[:, None].repeat(N, axis=1)
    return KX, KY


def _real_field(spec: np.ndarray) -> np.ndarray:
    """Real part of sum_k spec[k] exp(i k.x) on the N x N grid."""
    N = spec.shape[0]
    return np.real(np.fft.ifft2(spec)) * (N * N)


def geostrophic_field(N: int, k0: float, Ro: float, f: float, g: float, seed: int):
    """Balanced vortical flow (u, v, eta) with rms speed Ro * f."""
    rng = np.random.Generator(np.random.PCG64(seed))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(N, N))  # C order over the full lattice
    KX, KY = _int_wavenumbers(N)
    kk = np.sqrt(KX * KX + KY * KY)
    K = (N - 1) // 3
    inside = (np.abs(KX) <= K) & (np.abs(KY) <= K) & (kk > 0)
    amp = np.where(inside, np.sqrt(kk) * np.exp(-(kk * kk) / (2.0 * k0 * k0)), 0.0)
    psi_hat = amp * np.exp(1j * phase)
    u = _real_field(-1j * KY * psi_hat)
    v = _real_field(1j * KX * psi_hat)
    psi = _real_field(psi_hat)
    rms = np.sqrt(np.mean(u * u + v * v))
    scale = Ro * f / rms
    return u * scale, v * scale, (f / g) * psi * scale


def wave_field(N: int, k_lo: float, k_hi: float, f: float, g: float, H: float, seed: int):
    """Unit-amplitude band of Poincare waves (u, v, eta) at t = 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(N, N))
    KX, KY = _int_wavenumbers(N)
    k2 = KX * KX + KY * KY
    kk = np.sqrt(k2)
    band = (kk >= k_lo) & (kk <= k_hi) & (kk > 0)
    omega = np.sqrt(f * f + g * H * k2)
    c = np.where(band, np.exp(1j * phase), 0.0)
    safe = np.where(band, H * k2, 1.0)
    eta = _real_field(c)
    u = _real_field(c * (omega * KX + 1j * f * KY) / safe)
    v = _real_field(c * (omega * KY - 1j * f * KX) / safe)
    return u, v, eta


def linear_energy(u, v, eta, g: float, H: float) -> float:
    return 0.5 * float(np.mean(H * (u * u + v * v) + g * eta * eta))


def turbulence_plus_waves(N: int, *, k0: float, Ro: float, k_lo: float, k_hi: float,
                          ratio: float, seed_vortex: int, seed_wave: int,
                          f: float = 1.0, g: float = 1.0, H: float = 1.0):
    """Total-depth initial state (u, v, h) as float64 N x N arrays."""
    ug, vg, eg = geostrophic_field(N, k0, Ro, f, g, seed_vortex)
    uw, vw, ew = wave_field(N, k_lo, k_hi, f, g, H, seed_wave)
    ev = linear_energy(ug, vg, eg, g, H)
    ew_ = linear_energy(uw, vw, ew, g, H)
    a = np.sqrt(ratio * ev / ew_) if ew_ > 0 else 0.0
    u = ug + a * uw
    v = vg + a * vw
    h = H + eg + a * ew
    return np.ascontiguousarray(u), np.ascontiguousarray(v), np.ascontiguousarray(h)
