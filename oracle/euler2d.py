"""Two-dimensional incompressible inviscid flow with strategy 1 in two
discretisations (section 4.1, the vorticity test of eq. (4.2), and appendix B).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Dynamics: the vorticity equation dzeta/dt + (u + U0) . grad zeta = 0 with
u = (-dpsi/dy, dpsi/dx), lap psi = zeta (the k = 0 mode of psi is zero), on
[0, 2 pi)^2, pseudospectral with the 2/3-rule square mask (as the shallow-water
path) and Heun's method, as section 4.1 describes for this test.  (U0, V0) is
an optional uniform flow added to u (zero in the paper's test).

Strategy 1, pseudospectral: g~ = (t - tau) zeta~ by eq. (4.1),
dg~/dt + u . grad g~ = zeta, and the inverse lift map in the regular form
P = (t - tau)(x - Xi^{-1}), dP/dt + u . grad P = (t - tau) u (eq. (3.9)),
advanced in the same Heun stages.

Strategy 1, semi-Lagrangian (appendix B): after each step, at every grid
point X with departure point Y = X - dt u(X, t_{n+1}) (eq. (B.2)), the
trapezoidal update (B.4) of f~ (f = zeta) and (B.5) of Xi^{-1}, written for the
offset eta = X - Xi^{-1}(X).  With n = (t_n - tau)/dt and d = X - Y:

    f~_{n+1}(X) = [n f~_n(Y) + (f_n(Y) + f_{n+1}(X)) / 2] / (n + 1),
    eta_{n+1}(X) = [n eta_n(Y) + (n + 1/2) d] / (n + 1).

Values at Y come from the periodic bilinear (or cubic) interpolant at the small
offset -d.  At the end of the interval both give zeta~^L and eta; by material
conservation zeta~^L(x, tau) = zeta(x, tau + T) (eq. (4.2)).
"""

from __future__ import annotations

import numpy as np

from .lagmean import Grid, bilinear_periodic, cubic_periodic, irfft2, rfft2


class Euler2D:
    def __init__(self, N: int, dt: float, zeta0: np.ndarray, U0: float = 0.0, V0: float = 0.0,
                 interp: str = "bilinear"):
        self.G = Grid(N)
        self.N, self.dt, self.U0, self.V0 = N, dt, U0, V0
        self.gather = cubic_periodic if interp == "cubic" else bilinear_periodic
        k2 = self.G.KX ** 2 + self.G.KY ** 2
        self.inv_k2 = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
        self.Y = {"zeta": self.G.D * rfft2(np.asarray(zeta0, dtype=np.float64))}
        self.n = 0
        self.n_tau = 0
        self._zero_means()
        self.zeta_now = irfft2(self.Y["zeta"], N)

    def _zero_means(self):
        shape = self.Y["zeta"].shape
        for k in ("gtil", "P_x", "P_y"):
            self.Y[k] = np.zeros(shape, dtype=np.complex128)
        self.sl_f = np.zeros((self.N, self.N))
        self.sl_eta_x = np.zeros((self.N, self.N))
        self.sl_eta_y = np.zeros((self.N, self.N))

    def velocity(self, zeta_hat):
        """u = -dpsi/dy + U0, v = dpsi/dx + V0 with psi_hat = -zeta_hat / |k|^2."""
        G, N = self.G, self.N
        psi = -zeta_hat * self.inv_k2
        return irfft2(G.ddy(-psi), N) + self.U0, irfft2(G.ddx(psi), N) + self.V0

    def rhs(self, Y, s: float):
        G, N, D = self.G, self.N, self.G.D
        u, v = self.velocity(Y["zeta"])
        z = irfft2(Y["zeta"], N)
        zx, zy = irfft2(G.ddx(Y["zeta"]), N), irfft2(G.ddy(Y["zeta"]), N)
        R = {"zeta": -D * rfft2(u * zx + v * zy)}
        gx, gy = irfft2(G.ddx(Y["gtil"]), N), irfft2(G.ddy(Y["gtil"]), N)
        R["gtil"] = D * rfft2(z - (u * gx + v * gy))
        for comp, vel in (("P_x", u), ("P_y", v)):
            px, py = irfft2(G.ddx(Y[comp]), N), irfft2(G.ddy(Y[comp]), N)
            R[comp] = D * rfft2(s * vel - (u * px + v * py))
        return R

    def step(self, nsteps: int = 1):
        dt, N = self.dt, self.N
        for _ in range(nsteps):
            m = self.n - self.n_tau
            s0 = m * dt
            k1 = self.rhs(self.Y, s0)
            Y1 = {k: self.Y[k] + dt * k1[k] for k in self.Y}
            k2 = self.rhs(Y1, s0 + dt)
            self.Y = {k: self.Y[k] + 0.5 * dt * (k1[k] + k2[k]) for k in self.Y}
            # semi-Lagrangian strategy 1 with the velocity at t_{n+1}
            u, v = self.velocity(self.Y["zeta"])
            zeta_next = irfft2(self.Y["zeta"], N)
            d_x, d_y = dt * u, dt * v
            at = lambda F: self.gather(F, -d_x, -d_y, self.G.dx)
            f_Y, z_Y = at(self.sl_f), at(self.zeta_now)
            ex_Y, ey_Y = at(self.sl_eta_x), at(self.sl_eta_y)
            self.sl_f = (m * f_Y + 0.5 * (z_Y + zeta_next)) / (m + 1)
            self.sl_eta_x = (m * ex_Y + (m + 0.5) * d_x) / (m + 1)
            self.sl_eta_y = (m * ey_Y + (m + 0.5) * d_y) / (m + 1)
            self.zeta_now = zeta_next
            self.n += 1

    def begin_interval(self):
        self.n_tau = self.n
        self._zero_means()

    def end_interval(self):
        m = self.n - self.n_tau
        if m <= 0:
            raise RuntimeError("end_interval with no steps in the interval")
        T = m * self.dt
        N = self.N
        return {"zeta": irfft2(self.Y["zeta"], N),
                "PS_mean": irfft2(self.Y["gtil"], N) / T,
                "PS_eta_x": irfft2(self.Y["P_x"], N) / T, "PS_eta_y": irfft2(self.Y["P_y"], N) / T,
                "SL_mean": self.sl_f.copy(), "SL_eta_x": self.sl_eta_x.copy(), "SL_eta_y": self.sl_eta_y.copy()}
