"""Strategy 1 remapped to Lagrangian-mean positions (section 3.1, eq. (3.8)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Strategy 1 gives, on the grid of end-of-interval positions x, the mean f~^L(x)
and eta(x) = x - Xi^{-1}(x, tau + T), the offset to the mean position of the
particle found at x at the end of the interval.  Eq. (3.8) says
f~^L(x) = f-bar^L(Xi^{-1}(x)).  To get f-bar^L at a grid point y taken as a mean
position, find the end position x of the particle whose mean position is y:
x - eta(x) = y, i.e. the fixed point x = y + eta(x).  Then
f-bar^L(y) = f~^L(x), and d(y) = x - y = Xi(y) - y is the strategy-2
displacement xi(y) of the same particle.

The paper leaves the interpolation of the remap open (it warns that the mean
positions of a regular grid of x may cluster, section 5).  The reading here: the fixed point
is found by plain iteration d <- eta(y + d), starting from d = eta(y), with the
periodic bilinear interpolant of the strategy-2 gathers (section 4.2.1),
cells and weights from the small offset d / dx.  A point stops iterating once
an update moves d by at most tol * dx (max norm), or after max_iter updates.
The iteration contracts while the bilinear interpolant of eta has a Lipschitz
constant below one; its last update size is returned as the residual.
"""

from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from .lagmean import bilinear_periodic


def remap_s1(fields: Dict[str, np.ndarray], eta_x: np.ndarray, eta_y: np.ndarray, max_iter: int = 64,
             tol: float = 1e-13) -> Tuple[Dict[str, np.ndarray], np.ndarray, np.ndarray, np.ndarray]:
    """Remap strategy-1 means to Lagrangian-mean positions, eq. (3.8).

    fields: name -> f~^L on the grid (N x N, row-major [iy][ix]); eta_x, eta_y:
    x - Xi^{-1}(x).  Returns (f-bar^L per name at the grid points y, d_x, d_y =
    Xi(y) - y, residual per point in grid units)."""
    N = eta_x.shape[0]
    dx = 2.0 * np.pi / N
    d_x = np.array(eta_x, dtype=np.float64, copy=True)   # first guess x = y + eta(y)
    d_y = np.array(eta_y, dtype=np.float64, copy=True)
    residual = np.full(eta_x.shape, np.inf)
    active = np.ones(eta_x.shape, dtype=bool)
    for _ in range(max_iter):
        if not active.any():
            break
        n_x = bilinear_periodic(eta_x, d_x, d_y, dx)
        n_y = bilinear_periodic(eta_y, d_x, d_y, dx)
        step = np.maximum(np.abs(n_x - d_x), np.abs(n_y - d_y)) / dx
        d_x = np.where(active, n_x, d_x)
        d_y = np.where(active, n_y, d_y)
        residual = np.where(active, step, residual)
        active &= ~(step <= tol)
    out = {name: bilinear_periodic(np.asarray(f, dtype=np.float64), d_x, d_y, dx) for name, f in fields.items()}
    return out, d_x, d_y, residual
