"""Definition oracle: Lagrangian means by brute-force particle tracking.

TEST INFRASTRUCTURE ONLY.

Particles obey d phi/dt = u(phi, t) (the paper's eq. (2.1)).  Along each
trajectory the same classical RK4 (same dt, same stage times as ``lagmean``)
also integrates Phi = int phi ds and F = int f(phi, s) ds, so that over
(tau, tau + T):

* mean position  phi-bar^L = Phi / T                    (eq. (2.3))
* mean of f      F / T                                  (eqs. (2.4), (3.1))

and, for the mean of the momentum 1-form u . dx (appendix C, eq. (C.1)), the
label derivatives M = d phi / d a by the variational equation dM/dt = grad u M
(M = I at tau), their time integral (the mean map's Jacobian times T) and
int u_j M_ji ds (the pull-back phi_s^* (u . dx) integrated); eq. (C.1) then
reads (int M ds)^T tau-bar = int u_j M_j. ds at the particle's mean position.

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


def kinematic_velocity_gradient(p: Params, x: np.ndarray, y: np.ndarray, t: float):
    """(du/dx, du/dy, dv/dx, dv/dy) of the kinematic plane waves, analytically."""
    ux = np.zeros_like(x)
    uy = np.zeros_like(x)
    vx = np.zeros_like(x)
    vy = np.zeros_like(x)
    for w in p.waves:
        k2 = w.kx ** 2 + w.ky ** 2
        th = w.kx * x + w.ky * y - w.omega * t + w.phase
        c, s = np.cos(th), np.sin(th)
        a = w.A / (p.H * k2)
        # d/dtheta of (omega kx c - f ky s) is -(omega kx s + f ky c); likewise for v
        du = -a * (w.omega * w.kx * s + p.f * w.ky * c)
        dv = -a * (w.omega * w.ky * s - p.f * w.kx * c)
        ux, uy = ux + du * w.kx, uy + du * w.ky
        vx, vy = vx + dv * w.kx, vy + dv * w.ky
    return ux, uy, vx, vy


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


def track_momentum(p: Params, ax: np.ndarray, ay: np.ndarray, n_tau: int, nsteps: int) -> Dict[str, np.ndarray]:
    """Mean position, the mean map's Jacobian and the tracked mean of the
    momentum 1-form (eq. (C.1)) for particles with labels (ax, ay)."""
    assert p.mode == "kinematic"
    dt = p.dt
    z = np.zeros_like(ax, dtype=np.float64)
    # x, y, M_xx, M_xy, M_yx, M_yy (M_jk = d phi_j / d a_k), Phi_x, Phi_y,
    # int M (4 entries), int u_j M_jx, int u_j M_jy
    Y = [ax.astype(np.float64).copy(), ay.astype(np.float64).copy(), z + 1.0, z.copy(), z.copy(), z + 1.0,
         z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy(), z.copy()]

    def rhs(S, t):
        x, y, mxx, mxy, myx, myy = S[:6]
        u, v, _, _ = kinematic_fields(p, x, y, t)
        ux, uy, vx, vy = kinematic_velocity_gradient(p, x, y, t)
        return [u, v,
                ux * mxx + uy * myx, ux * mxy + uy * myy, vx * mxx + vy * myx, vx * mxy + vy * myy,
                x, y, mxx, mxy, myx, myy, u * mxx + v * myx, u * mxy + v * myy]

    for n in range(n_tau, n_tau + nsteps):
        ks = []
        for i, c in enumerate(RK4_C):
            Si = Y if i == 0 else [a + (c * dt) * k for a, k in zip(Y, ks[-1])]
            ks.append(rhs(Si, (n + c) * dt))
        Y = [a + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4) for a, k1, k2, k3, k4 in zip(Y, *ks)]
    T = nsteps * dt
    Ixx, Ixy, Iyx, Iyy, Rx, Ry = Y[8:14]
    # (int M)^T tau = R:  [Ixx Iyx; Ixy Iyy] tau = R
    det = Ixx * Iyy - Iyx * Ixy
    tx = (Iyy * Rx - Iyx * Ry) / det
    ty = (-Ixy * Rx + Ixx * Ry) / det
    return {"xbar": Y[6] / T, "ybar": Y[7] / T, "mom_x": tx, "mom_y": ty}


def _s2_labels(p: Params, n_tau: int, nsteps: int, tol: float, max_iter: int):
    """Labels whose mean positions are the grid points (fixed-point iteration)."""
    N = p.N
    dx = 2.0 * math.pi / N
    gx = np.broadcast_to((np.arange(N) * dx)[None, :], (N, N)).copy()
    gy = np.broadcast_to((np.arange(N) * dx)[:, None], (N, N)).copy()
    ax, ay = gx.copy(), gy.copy()
    for _ in range(max_iter):
        r = track(p, ax, ay, n_tau, nsteps, ())
        ex = _wrap(gx - r["xbar"])
        ey = _wrap(gy - r["ybar"])
        ax += ex
        ay += ey
        if max(np.max(np.abs(ex)), np.max(np.abs(ey))) < tol:
            break
    return ax, ay


def momentum_mean_by_tracking(p: Params, n_tau: int, nsteps: int, tol: float = 1e-13,
                              max_iter: int = 200) -> Dict[str, np.ndarray]:
    """Strategy-2 mean of the momentum 1-form on the grid (mean positions) by
    tracking, eq. (C.1): 'S2_mom_x', 'S2_mom_y'."""
    ax, ay = _s2_labels(p, n_tau, nsteps, tol, max_iter)
    r = track_momentum(p, ax, ay, n_tau, nsteps)
    return {"S2_mom_x": r["mom_x"], "S2_mom_y": r["mom_y"]}


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
