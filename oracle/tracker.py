"""Definition oracle: Lagrangian means by brute-force particle tracking.

TEST INFRASTRUCTURE ONLY.

Particles obey d phi/dt = u(phi, t) (the paper's eq. (2.1)).  Along each
trajectory the same classical RK4 (same dt, same stage times as ``lagmean``)
also integrates Phi = int phi ds and F = int f(phi, s) ds, so that over
(tau, tau + T):

* mean position  phi-bar^L = Phi / T                    (eq. (2.3))
* mean of f      F / T                                  (eqs. (2.4), (3.1))

Strategy 2's outputs at a grid point x are those of the particle whose mean
position is x (f-bar^L(x) = F/T, xi(x) = phi(tau+T) - x); strategy 1's outputs
at x are those of the particle that ends at x (f~^L(x) = F/T,
eta(x) = x - Phi/T, i.e. x - Xi^{-1}(x)).  Both labels are found by
fixed-point iteration on the label.

Only the kinematic driver is supported: u, v, h are the analytic plane waves of
``lagmean.Params`` evaluated exactly at any point, so the only discretisation
error left here is RK4's in time.
"""

from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np

from .lagmean import Params, RK4_C


def kinematic_fields(p: Params, x: np.ndarray, y: np.ndarray, t: float):
    u = np.full_like(x, p.U0)
    v = np.full_like(x, p.V0)
    h = np.full_like(x, p.H)
    z = np.zeros_like(x)
    for w in p.waves:
        k2 = w.kx ** 2 + w.ky ** 2
        th = w.kx * x + w.ky * y - w.omega * t + w.phase
        c, s = np.cos(th), np.sin(th)
        u = u + w.A * (w.omega * w.kx * c - p.f * w.ky * s) / (p.H * k2)
        v = v + w.A * (w.omega * w.ky * c + p.f * w.kx * s) / (p.H * k2)
        h = h + w.A * c
        z = z + w.A * p.f * c / p.H
    return u, v, h, z


def _field_values(p: Params, names: Sequence[str], u, v, h, z):
    out = []
    for m in names:
        if m == "h":
            out.append(h)
        elif m == "zeta":
            out.append(z)
        elif m == "q":
            out.append((p.f + z) / h)
        elif m == "u":
            out.append(u)
        elif m == "v":
            out.append(v)
        elif m == "one":
            out.append(np.ones_like(h))
        else:
            raise ValueError(m)
    return out


def track(p: Params, ax: np.ndarray, ay: np.ndarray, n_tau: int, nsteps: int,
          names: Sequence[str]) -> Dict[str, np.ndarray]:
    """Advance particles with labels (ax, ay) at t = n_tau dt over nsteps steps."""
    assert p.mode == "kinematic"
    dt = p.dt
    m = len(names)
    # state: x, y, Phi_x, Phi_y, F_1..F_m  (positions are not wrapped)
    Y = [ax.astype(np.float64).copy(), ay.astype(np.float64).copy(),
         np.zeros_like(ax, dtype=np.float64), np.zeros_like(ax, dtype=np.float64)]
    Y += [np.zeros_like(ax, dtype=np.float64) for _ in range(m)]

    def rhs(S, t):
        u, v, h, z = kinematic_fields(p, S[0], S[1], t)
        return [u, v, S[0], S[1]] + _field_values(p, names, u, v, h, z)

    for n in range(n_tau, n_tau + nsteps):
        ks = []
        for i, c in enumerate(RK4_C):
            if i == 0:
                Si = Y
            else:
                Si = [a + (c * dt) * k for a, k in zip(Y, ks[-1])]
            ks.append(rhs(Si, (n + c) * dt))
        Y = [a + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
             for a, k1, k2, k3, k4 in zip(Y, *ks)]
    T = nsteps * dt
    out = {"x_end": Y[0], "y_end": Y[1], "xbar": Y[2] / T, "ybar": Y[3] / T}
    for j, name in enumerate(names):
        out[name] = Y[4 + j] / T
    return out


def _wrap(d: np.ndarray) -> np.ndarray:
    return (d + math.pi) % (2.0 * math.pi) - math.pi


def means_by_tracking(p: Params, n_tau: int, nsteps: int, names: Sequence[str],
                      tol: float = 1e-13, max_iter: int = 200) -> Dict[str, np.ndarray]:
    """Strategy-1 and strategy-2 outputs on the N x N grid by tracking."""
    N = p.N
    dx = 2.0 * math.pi / N
    gx = np.broadcast_to((np.arange(N) * dx)[None, :], (N, N)).copy()
    gy = np.broadcast_to((np.arange(N) * dx)[:, None], (N, N)).copy()
    out: Dict[str, np.ndarray] = {}

    # strategy 2: label whose mean position is the grid point
    ax, ay = gx.copy(), gy.copy()
    for _ in range(max_iter):
        r = track(p, ax, ay, n_tau, nsteps, names)
        ex = _wrap(gx - r["xbar"])
        ey = _wrap(gy - r["ybar"])
        ax += ex
        ay += ey
        if max(np.max(np.abs(ex)), np.max(np.abs(ey))) < tol:
            break
    r = track(p, ax, ay, n_tau, nsteps, names)
    out["S2_xi_x"] = r["x_end"] - (r["xbar"])
    out["S2_xi_y"] = r["y_end"] - (r["ybar"])
    for name in names:
        out[f"S2_mean:{name}"] = r[name]

    # strategy 1: label that ends at the grid point
    ax, ay = gx.copy(), gy.copy()
    for _ in range(max_iter):
        r = track(p, ax, ay, n_tau, nsteps, names)
        ex = _wrap(gx - r["x_end"])
        ey = _wrap(gy - r["y_end"])
        ax += ex
        ay += ey
        if max(np.max(np.abs(ex)), np.max(np.abs(ey))) < tol:
            break
    r = track(p, ax, ay, n_tau, nsteps, names)
    out["S1_eta_x"] = r["x_end"] - r["xbar"]
    out["S1_eta_y"] = r["y_end"] - r["ybar"]
    for name in names:
        out[f"S1_mean:{name}"] = r[name]
    return out
