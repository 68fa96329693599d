"""Plain float64 oracle of the coupled shallow-water / Lagrangian-mean stepper.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written for clarity,
not speed: every array is a full N x N (physical) or N x (N/2+1) (spectral,
``numpy.fft.rfft2`` convention, unnormalised forward) float64/complex128 array.

What is computed (the paper: Kafiabad & Vanneste, "Computing Lagrangian
means"):

* Time average over successive intervals (tau, tau + T), tau = n T, each interval
  independent (section 3, after eq. (3.3)).
* Strategy 1 (section 3.1, numerics section 4.1): the partial mean f~ of eq. (3.5)
  is integrated in the form g~ = (t - tau) f~ of eq. (4.1),
      d g~/dt + u . grad g~ = f,   g~(tau) = 0,   f~^L = g~(tau+T) / T.
  The inverse lift map Xi^{-1} of eq. (3.9) is integrated in the same spirit as
  P = (t - tau) (x - Xi^{-1}(x, t)), which is periodic and regular at t = tau:
  along a trajectory P = (t-tau) phi - int_tau^t phi ds, so DP/Dt = (t - tau) u,
      dP/dt + u . grad P = (t - tau) u,   P(tau) = 0,
  and at the end eta = x - Xi^{-1} = P / T.  (Substituting Xi^{-1} = x - P/(t-tau)
  into eq. (3.9) gives the same equation.)
* Strategy 2 (section 3.2, numerics section 4.2): the displacement
  xi = Xi - x (eq. (4.4)) and g = (t - tau) f-bar obey eqs. (4.5a,b) with the
  partial-mean velocity u-bar = xi / (t - tau) (eq. (3.11)),
      d xi/dt + w . grad xi = u(x + xi) - w,   d g/dt + w . grad g = f(x + xi),
  w = xi / (t - tau), xi(tau) = 0, g(tau) = 0, f-bar^L = g(tau+T) / T.
  At t = tau, where xi / (t - tau) is 0/0, w takes its limit u(x, tau) / 2
  (the partial mean position moves at half the particle velocity initially).
  u and f at x + xi are bilinear interpolants (section 4.2.1), periodic.
* Eulerian mean: dE/dt = f, E(tau) = 0, E-bar = E(tau+T) / T.
* Dynamics: rotating shallow water, section 4.2 eq. (4.6), in dimensional
  vector-invariant form with total depth h,
      du/dt = (zeta) v + f v - d/dx (K + g h),
      dv/dt = -(zeta) u - f u - d/dy (K + g h),
      dh/dt = -d/dx (h u) - d/dy (h v),
  K = (u^2 + v^2)/2, zeta = dv/dx - du/dy, plus -nu8 |k|^8 on u, v, h.
* Space: Fourier pseudospectral on [0, 2 pi)^2 with the 2/3-rule square mask
  |kx|, |ky| <= floor((N-1)/3) (sections 4.1, 4.2.1) applied to the initial state
  and to every right-hand side; products are formed on the N x N grid.
* Time: one classical RK4 over all fields with a shared dt; stage times
  t_n + c_i dt, c = (0, 1/2, 1/2, 1); the time since the interval start is
  s = (n - n_tau + c_i) dt from integers.

Two alternative drivers for u, v, h:
* ``mode = "dynamic"``: the shallow-water equations above;
* ``mode = "kinematic"``: u, v, h prescribed analytically as a uniform flow plus
  linear Poincare plane waves (section 4.2.1, eq. (4.8), any direction), which
  admits exact particle trajectories (the pins in ``closed``).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Sequence, Tuple

import numpy as np
import scipy.fft as sfft

WORKERS = 1  # threads the FFT library may use; the benchmark raises it


def set_workers(n: int) -> None:
    global WORKERS
    WORKERS = max(1, int(n))


def rfft2(a: np.ndarray) -> np.ndarray:
    return sfft.rfft2(a, workers=WORKERS)


def irfft2(a: np.ndarray, N: int) -> np.ndarray:
    return sfft.irfft2(a, s=(N, N), workers=WORKERS)


# --------------------------------------------------------------------------
# averaged fields f(u, v, h, zeta); the product path averages h and zeta
# --------------------------------------------------------------------------

def _f_h(u, v, h, z, p):
    # the depth is averaged as its anomaly h - H; H is added to the outputs
    # (the average is linear in f and exact for constants, eq. (2.4)), which
    # keeps the accumulators free of the large constant part
    return h - p.H


def _f_zeta(u, v, h, z, p):
    return z


def _f_q(u, v, h, z, p):  # potential vorticity (f + zeta)/h, materially conserved
    return (p.f + z) / h


def _f_u(u, v, h, z, p):
    return u


def _f_v(u, v, h, z, p):
    return v


def _f_one(u, v, h, z, p):
    return np.ones_like(h)


BUILTIN_FIELDS: Dict[str, Callable] = {
    "h": _f_h, "zeta": _f_zeta, "q": _f_q, "u": _f_u, "v": _f_v, "one": _f_one,
}


def field_offset(name: str, p) -> float:
    """Constant removed from an averaged field before accumulation."""
    return p.H if name == "h" else 0.0


@dataclass
class PlaneWave:
    """Linear Poincare wave h' = A cos(theta), theta = kx x + ky y - omega t + phase,
    with the linear shallow-water polarisation (section 4.2.1, eq. (4.8), rotated)."""
    kx: float
    ky: float
    A: float
    omega: float
    phase: float = 0.0


@dataclass
class Params:
    N: int
    dt: float
    f: float = 1.0
    g: float = 1.0
    H: float = 1.0
    nu8: float = 0.0
    fields: Sequence[str] = ("h", "zeta")
    mode: str = "dynamic"                      # or "kinematic"
    waves: List[PlaneWave] = field(default_factory=list)   # kinematic mode
    U0: float = 0.0                            # kinematic uniform flow
    V0: float = 0.0
    interp: str = "bilinear"                   # strategy-2 gathers: "bilinear" or "cubic"
    momentum: bool = False                     # strategy-2 mean of the momentum 1-form (appendix C)


class Grid:
    """Grid, integer wavenumbers and the 2/3-rule mask for the rfft2 layout."""

    def __init__(self, N: int):
        self.N = N
        self.dx = 2.0 * math.pi / N
        x = np.arange(N) * self.dx
        self.X = np.broadcast_to(x[None, :], (N, N))
        self.Y = np.broadcast_to(x[:, None], (N, N))
        kx = np.arange(N // 2 + 1, dtype=np.float64)
        ky = np.fft.fftfreq(N, d=1.0 / N)
        self.KX = np.broadcast_to(kx[None, :], (N, N // 2 + 1))
        self.KY = np.broadcast_to(ky[:, None], (N, N // 2 + 1))
        self.Kc = (N - 1) // 3
        self.D = ((np.abs(self.KX) <= self.Kc) & (np.abs(self.KY) <= self.Kc)).astype(np.float64)
        k2 = self.KX ** 2 + self.KY ** 2
        self.K8 = k2 ** 4

    def ddx(self, a_hat):
        return 1j * self.KX * a_hat

    def ddy(self, a_hat):
        return 1j * self.KY * a_hat


def bilinear_periodic(F: np.ndarray, xi_x: np.ndarray, xi_y: np.ndarray, dx: float) -> np.ndarray:
    """Bilinear interpolant of the periodic grid field F at x + xi for every grid
    point x (section 4.2.1).  Cell indices and weights come from the small offset
    xi/dx, not from an absolute position."""
    N = F.shape[0]
    ox = xi_x / dx
    oy = xi_y / dx
    fx = np.floor(ox)
    fy = np.floor(oy)
    ax = ox - fx
    ay = oy - fy
    jx = np.arange(N)[None, :]
    jy = np.arange(N)[:, None]
    ix0 = (jx + fx.astype(np.int64)) % N
    iy0 = (jy + fy.astype(np.int64)) % N
    ix1 = (ix0 + 1) % N
    iy1 = (iy0 + 1) % N
    return ((1.0 - ax) * (1.0 - ay) * F[iy0, ix0] + ax * (1.0 - ay) * F[iy0, ix1]
            + (1.0 - ax) * ay * F[iy1, ix0] + ax * ay * F[iy1, ix1])


def cubic_periodic(F: np.ndarray, xi_x: np.ndarray, xi_y: np.ndarray, dx: float) -> np.ndarray:
    """Tensor-product cubic (4-point Lagrange) interpolant of the periodic grid
    field F at x + xi for every grid point x: with o = xi/dx, i0 = floor(o) and
    a = o - i0, the nodes i0-1 .. i0+2 carry the Lagrange weights
    L(-1) = -a(a-1)(a-2)/6, L(0) = (a+1)(a-1)(a-2)/2, L(1) = -(a+1)a(a-2)/2,
    L(2) = (a+1)a(a-1)/6.  Exact for cubics, continuous across cells, error
    O(dx^4) for smooth fields.  Cells and weights from the small offset xi/dx."""
    N = F.shape[0]
    ox = xi_x / dx
    oy = xi_y / dx
    fx = np.floor(ox)
    fy = np.floor(oy)
    ax = ox - fx
    ay = oy - fy

    def weights(a):
        return (-a * (a - 1.0) * (a - 2.0) / 6.0, (a + 1.0) * (a - 1.0) * (a - 2.0) / 2.0,
                -(a + 1.0) * a * (a - 2.0) / 2.0, (a + 1.0) * a * (a - 1.0) / 6.0)

    wx, wy = weights(ax), weights(ay)
    jx = np.arange(N)[None, :]
    jy = np.arange(N)[:, None]
    ix0 = jx + fx.astype(np.int64)
    iy0 = jy + fy.astype(np.int64)
    out = np.zeros(F.shape)
    for j in range(4):
        row = np.zeros(F.shape)
        iy = (iy0 + j - 1) % N
        for i in range(4):
            row += wx[i] * F[iy, (ix0 + i - 1) % N]
        out += wy[j] * row
    return out


RK4_C = (0.0, 0.5, 0.5, 1.0)


class Run:
    """One run: dynamics state plus strategy-1, strategy-2 and Eulerian state.

    State entries (spectral, rfft2 layout): 'u','v','h' (dynamic mode only),
    'xi_x','xi_y','gbar:<f>' (strategy 2), 'gtil:<f>','P_x','P_y' (strategy 1),
    'E:<f>' (Eulerian accumulator), for every averaged field name <f>.  The
    accumulators of 'h' integrate the anomaly h - H (see ``field_offset``).
    """

    def __init__(self, p: Params, u0=None, v0=None, h0=None):
        self.p = p
        self.grid = Grid(p.N)
        self.fields = list(p.fields)
        self.ffun = {name: BUILTIN_FIELDS[name] for name in self.fields}
        self.n = 0
        self.n_tau = 0
        self.Y: Dict[str, np.ndarray] = {}
        if p.mode == "dynamic":
            for name, a in (("u", u0), ("v", v0), ("h", h0)):
                self.Y[name] = self.grid.D * rfft2(np.asarray(a, dtype=np.float64))
        elif p.mode != "kinematic":
            raise ValueError(p.mode)
        self._zero_means()
        self.outputs: Dict[str, np.ndarray] = {}
        self.T = None

    # ------------------------------------------------------------------ state
    def _mean_keys(self):
        keys = ["xi_x", "xi_y", "P_x", "P_y"]
        if self.p.momentum:
            keys += ["gmom_x", "gmom_y"]
        for m in self.fields:
            keys += [f"gbar:{m}", f"gtil:{m}", f"E:{m}"]
        return keys

    def _zero_means(self):
        shape = (self.p.N, self.p.N // 2 + 1)
        for k in self._mean_keys():
            self.Y[k] = np.zeros(shape, dtype=np.complex128)

    def physical(self, key: str) -> np.ndarray:
        return irfft2(self.Y[key], self.p.N)

    # ------------------------------------------------------------------ driver fields
    def _kinematic(self, t: float):
        p, G = self.p, self.grid
        u = np.full((p.N, p.N), p.U0)
        v = np.full((p.N, p.N), p.V0)
        h = np.full((p.N, p.N), p.H)
        z = np.zeros((p.N, p.N))
        for w in p.waves:
            k2 = w.kx ** 2 + w.ky ** 2
            th = w.kx * G.X + w.ky * G.Y - w.omega * t + w.phase
            c, s = np.cos(th), np.sin(th)
            u = u + w.A * (w.omega * w.kx * c - p.f * w.ky * s) / (p.H * k2)
            v = v + w.A * (w.omega * w.ky * c + p.f * w.kx * s) / (p.H * k2)
            h = h + w.A * c
            z = z + w.A * p.f * c / p.H
        return u, v, h, z

    # ------------------------------------------------------------------ right-hand side
    def rhs(self, Y: Dict[str, np.ndarray], s: float, t: float) -> Dict[str, np.ndarray]:
        p, G, N = self.p, self.grid, self.p.N
        D = G.D
        R: Dict[str, np.ndarray] = {}

        if p.mode == "dynamic":
            u = irfft2(Y["u"], N)
            v = irfft2(Y["v"], N)
            h = irfft2(Y["h"], N)
            z = irfft2(G.ddx(Y["v"]) - G.ddy(Y["u"]), N)
            K = 0.5 * (u * u + v * v)
            F_zv = rfft2(z * v)
            F_zu = rfft2(z * u)
            F_B = p.g * Y["h"] + rfft2(K)          # Bernoulli function K + g h
            F_hu = rfft2(h * u)
            F_hv = rfft2(h * v)
            R["u"] = D * (F_zv + p.f * Y["v"] - G.ddx(F_B)) - p.nu8 * G.K8 * Y["u"]
            R["v"] = D * (-F_zu - p.f * Y["u"] - G.ddy(F_B)) - p.nu8 * G.K8 * Y["v"]
            R["h"] = D * (-G.ddx(F_hu) - G.ddy(F_hv)) - p.nu8 * G.K8 * Y["h"]
        else:
            u, v, h, z = self._kinematic(t)

        fval = {m: self.ffun[m](u, v, h, z, p) for m in self.fields}

        # strategy 2: displacement xi and g-bar, eqs. (4.5a,b)
        xi_x = irfft2(Y["xi_x"], N)
        xi_y = irfft2(Y["xi_y"], N)
        if s > 0.0:
            wx, wy = xi_x / s, xi_y / s
        else:
            wx, wy = 0.5 * u, 0.5 * v
        gather = cubic_periodic if p.interp == "cubic" else bilinear_periodic
        u_at = gather(u, xi_x, xi_y, G.dx)
        v_at = gather(v, xi_x, xi_y, G.dx)
        for comp, src in (("xi_x", u_at), ("xi_y", v_at)):
            dxi_dx = irfft2(G.ddx(Y[comp]), N)
            dxi_dy = irfft2(G.ddy(Y[comp]), N)
            R[comp] = D * rfft2(src - (wx if comp == "xi_x" else wy) - (wx * dxi_dx + wy * dxi_dy))
        for m in self.fields:
            key = f"gbar:{m}"
            f_at = gather(fval[m], xi_x, xi_y, G.dx)
            dg_dx = irfft2(G.ddx(Y[key]), N)
            dg_dy = irfft2(G.ddy(Y[key]), N)
            R[key] = D * rfft2(f_at - (wx * dg_dx + wy * dg_dy))
        if p.momentum:
            # appendix C, eq. (C.4) for the 1-form u . dx in the g-bar form of
            # eq. (4.5b): with g = (t - tau) tau-bar and u-bar = w,
            #   dg_i/dt + w_j d_j g_i + g_j d_i w_j = u_j(x + xi) (delta_ij + d_i xi_j)
            # (the pull-back by Xi = x + xi on the right).  At t = tau, g = 0, so
            # the d_i w_j term vanishes there and is only formed for s > 0.
            dxi = {(c, d): irfft2((G.ddx if d == "x" else G.ddy)(Y[f"xi_{c}"]), N)
                   for c in ("x", "y") for d in ("x", "y")}   # dxi[(j, i)] = d_i xi_j
            gm = {c: irfft2(Y[f"gmom_{c}"], N) for c in ("x", "y")}
            for i in ("x", "y"):
                key = f"gmom_{i}"
                src = u_at * ((1.0 if i == "x" else 0.0) + dxi[("x", i)]) \
                    + v_at * ((1.0 if i == "y" else 0.0) + dxi[("y", i)])
                dg_dx = irfft2(G.ddx(Y[key]), N)
                dg_dy = irfft2(G.ddy(Y[key]), N)
                rhs_i = src - (wx * dg_dx + wy * dg_dy)
                if s > 0.0:
                    rhs_i = rhs_i - (gm["x"] * dxi[("x", i)] + gm["y"] * dxi[("y", i)]) / s
                R[key] = D * rfft2(rhs_i)

        # strategy 1: g-tilde, eq. (4.1), and P for the inverse lift map, eq. (3.9)
        for m in self.fields:
            key = f"gtil:{m}"
            dg_dx = irfft2(G.ddx(Y[key]), N)
            dg_dy = irfft2(G.ddy(Y[key]), N)
            R[key] = D * rfft2(fval[m] - (u * dg_dx + v * dg_dy))
        for comp, vel in (("P_x", u), ("P_y", v)):
            dP_dx = irfft2(G.ddx(Y[comp]), N)
            dP_dy = irfft2(G.ddy(Y[comp]), N)
            R[comp] = D * rfft2(s * vel - (u * dP_dx + v * dP_dy))

        # Eulerian accumulator
        for m in self.fields:
            R[f"E:{m}"] = D * rfft2(fval[m])
        return R

    # ------------------------------------------------------------------ time stepping
    def step(self, nsteps: int = 1) -> None:
        dt = self.p.dt
        for _ in range(nsteps):
            Y0 = self.Y
            ks = []
            for i, c in enumerate(RK4_C):
                if i == 0:
                    Yi = Y0
                else:
                    Yi = {k: Y0[k] + (c * dt) * ks[-1][k] for k in Y0}
                s = (self.n - self.n_tau + c) * dt
                t = (self.n + c) * dt
                ks.append(self.rhs(Yi, s, t))
            self.Y = {k: Y0[k] + (dt / 6.0) * (ks[0][k] + 2.0 * ks[1][k] + 2.0 * ks[2][k] + ks[3][k])
                      for k in Y0}
            self.n += 1

    def begin_interval(self) -> None:
        self.n_tau = self.n
        self._zero_means()

    def end_interval(self) -> Dict[str, np.ndarray]:
        nsteps = self.n - self.n_tau
        if nsteps <= 0:
            raise RuntimeError("end_interval with no steps in the interval")
        T = nsteps * self.p.dt
        N = self.p.N
        out = {
            "S2_xi_x": irfft2(self.Y["xi_x"], N),
            "S2_xi_y": irfft2(self.Y["xi_y"], N),
            "S1_eta_x": irfft2(self.Y["P_x"], N) / T,
            "S1_eta_y": irfft2(self.Y["P_y"], N) / T,
        }
        if self.p.momentum:
            out["S2_mom_x"] = irfft2(self.Y["gmom_x"], N) / T
            out["S2_mom_y"] = irfft2(self.Y["gmom_y"], N) / T
        for m in self.fields:
            c = field_offset(m, self.p)
            out[f"S2_mean:{m}"] = irfft2(self.Y[f"gbar:{m}"], N) / T + c
            out[f"S1_mean:{m}"] = irfft2(self.Y[f"gtil:{m}"], N) / T + c
            out[f"E_mean:{m}"] = irfft2(self.Y[f"E:{m}"], N) / T + c
        self.T = T
        self.outputs = out
        return out

    def run_intervals(self, steps_per_interval: int, n_intervals: int):
        results = []
        for _ in range(n_intervals):
            self.begin_interval()
            self.step(steps_per_interval)
            results.append(self.end_interval())
        return results

    def dynamics_physical(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        N = self.p.N
        return irfft2(self.Y["u"], N), irfft2(self.Y["v"], N), irfft2(self.Y["h"], N)


def relative_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 over the grid; absolute max error when ||b|| < 1e-14."""
    nb = float(np.linalg.norm(b))
    if nb < 1e-14:
        return float(np.max(np.abs(a - b)))
    return float(np.linalg.norm(a - b)) / nb
