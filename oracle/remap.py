"""Strategy 1 remapped to Lagrangian-mean positions (section 3.1, eq. (3.8)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Strategy 1 gives, on the grid of end-of-interval positions x, the mean f~^L(x)
and eta(x) = x - Xi^{-1}(x, tau + T), the offset to the mean position of the
particle found at x at the end of the interval.  Eq. (3.8) says
f~^L(x) = f-bar^L(Xi^{-1}(x)).  To get f-bar^L at a grid point y taken as a mean
position, find the end position x of the particle whose mean position is y:

    x - eta(x) = y,   then  f-bar^L(y) = f~^L(x),  d(y) = x - y = Xi(y) - y

(d is the strategy-2 displacement xi(y) of the same particle).

The paper leaves the interpolation of the remap open and warns that the mean
positions of a regular grid of x may cluster (section 5).  The reading here:
eta and f~^L are the periodic bilinear interpolants of their grid values (the
interpolant of the strategy-2 gathers, section 4.2.1), and the equation is
solved exactly, cell by cell.  On the end-position cell with corners
(ix, iy) .. (ix + 1, iy + 1) (grid units) the map x -> x - eta(x) is the
bilinear patch through the four corner mean positions; every grid point y that
the patch covers is located by inverting the patch (closed form, then two
Newton steps), which gives the end position x = (ix + s, iy + t) and, with the
same weights, f~^L(x).  Plain fixed-point iteration x <- y + eta(x) solves the
same equation but stops contracting where eta varies by more than a cell per
cell, which the workloads reach within one interval; the patch inversion has
no such limit.  Where the mean map folds (a point covered by several patches)
the patch of the lowest cell index (iy N + ix) is taken; a point covered by no
patch (only possible through a cell whose patch spans more than max_extent
cells, or lies more than 1e7 cells away, which is then skipped) gets NaN and
an infinite residual.
"""

from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

EPS = 1e-12  # tolerance of the inside test in the patch coordinates s, t


def _cross(ax, ay, bx, by):
    return ax * by - ay * bx


def invert_patch(p00, p10, p01, p11, Yx, Yy):
    """Patch coordinates (s, t) with p(s, t) = Y for the bilinear patch
    p(s, t) = p00 (1-s)(1-t) + p10 s (1-t) + p01 (1-s) t + p11 s t (points as
    (x, y) pairs of arrays).  Returns (s, t, ok); of the two roots of the
    quadratic the one closer to the unit square is taken."""
    ax, ay = p00
    bx, by = p10[0] - ax, p10[1] - ay
    cx, cy = p01[0] - ax, p01[1] - ay
    dx_, dy_ = p11[0] - p10[0] - p01[0] + ax, p11[1] - p10[1] - p01[1] + ay
    qx, qy = Yx - ax, Yy - ay
    # q = b s + (c + d s) t; crossing with (c + d s) removes t:
    # (b x d) s^2 + (b x c - q x d) s - q x c = 0
    A = _cross(bx, by, dx_, dy_)
    B = _cross(bx, by, cx, cy) - _cross(qx, qy, dx_, dy_)
    C = -_cross(qx, qy, cx, cy)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        scale = np.abs(B) + 1e-300
        lin = np.abs(A) <= 1e-14 * scale
        disc = B * B - 4.0 * A * C
        sq = np.sqrt(np.maximum(disc, 0.0))
        qq = -0.5 * (B + np.copysign(sq, B))
        r1 = np.where(lin, -C / B, qq / A)
        r2 = np.where(lin, -C / B, C / qq)

        def t_of(s):
            wx, wy = cx + dx_ * s, cy + dy_ * s
            return ((qx - bx * s) * wx + (qy - by * s) * wy) / (wx * wx + wy * wy)

        t1, t2 = t_of(r1), t_of(r2)
        dist = lambda s, t: np.maximum(np.maximum(-s, s - 1.0), np.maximum(-t, t - 1.0))
        pick1 = ~(dist(r2, t2) < dist(r1, t1))
        s = np.where(pick1, r1, r2)
        t = np.where(pick1, t1, t2)
        # two Newton steps on the bilinear system
        for _ in range(2):
            rx = ax + bx * s + cx * t + dx_ * s * t - Yx
            ry = ay + by * s + cy * t + dy_ * s * t - Yy
            j11, j12 = bx + dx_ * t, cx + dx_ * s
            j21, j22 = by + dy_ * t, cy + dy_ * s
            det = j11 * j22 - j12 * j21
            s = s - (j22 * rx - j12 * ry) / det
            t = t - (-j21 * rx + j11 * ry) / det
        ok = np.isfinite(s) & np.isfinite(t) & (lin | (disc >= 0.0))
    return s, t, ok


def remap_s1(fields: Dict[str, np.ndarray], eta_x: np.ndarray, eta_y: np.ndarray,
             max_extent: int = 64) -> Tuple[Dict[str, np.ndarray], np.ndarray, np.ndarray, np.ndarray]:
    """Remap strategy-1 means to Lagrangian-mean positions, eq. (3.8).

    fields: name -> f~^L on the grid (N x N, row-major [iy][ix]); eta_x, eta_y:
    x - Xi^{-1}(x).  Returns (f-bar^L per name at the grid points y, d_x, d_y =
    Xi(y) - y, residual |p(s, t) - y| per point in grid units)."""
    N = eta_x.shape[0]
    h = 2.0 * np.pi / N
    ex, ey = eta_x / h, eta_y / h
    IY, IX = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")

    def corner(ox, oy):
        jx, jy = (IX + ox) % N, (IY + oy) % N
        return (IX + ox - ex[jy, jx], IY + oy - ey[jy, jx]), (jy, jx)

    p00, c00 = corner(0, 0)
    p10, c10 = corner(1, 0)
    p01, c01 = corner(0, 1)
    p11, c11 = corner(1, 1)
    xs = np.stack([p00[0], p10[0], p01[0], p11[0]])
    ys = np.stack([p00[1], p10[1], p01[1], p11[1]])
    lo_x, hi_x = np.ceil(xs.min(0) - EPS), np.floor(xs.max(0) + EPS)
    lo_y, hi_y = np.ceil(ys.min(0) - EPS), np.floor(ys.max(0) + EPS)
    usable = ((hi_x - lo_x <= max_extent) & (hi_y - lo_y <= max_extent)
              & (np.abs(lo_x) < 1e7) & (np.abs(hi_x) < 1e7) & (np.abs(lo_y) < 1e7) & (np.abs(hi_y) < 1e7))
    ext_x = int(np.max(np.where(usable, hi_x - lo_x, 0)))
    ext_y = int(np.max(np.where(usable, hi_y - lo_y, 0)))
    cell = IY * N + IX
    BIG = np.iinfo(np.int64).max
    best = np.full(N * N, BIG, dtype=np.int64)
    cands = []
    for oy in range(ext_y + 1):
        for ox in range(ext_x + 1):
            Yx, Yy = lo_x + ox, lo_y + oy
            valid = usable & (Yx <= hi_x) & (Yy <= hi_y)
            s, t, ok = invert_patch(p00, p10, p01, p11, Yx, Yy)
            inside = valid & ok & (s >= -EPS) & (s <= 1 + EPS) & (t >= -EPS) & (t <= 1 + EPS)
            if not inside.any():
                continue
            tgt = ((Yy.astype(np.int64) % N) * N + (Yx.astype(np.int64) % N))[inside]
            np.minimum.at(best, tgt, cell[inside])
            cands.append((tgt, cell[inside], s[inside], t[inside], Yx[inside], Yy[inside]))
    d_x = np.full(N * N, np.nan)
    d_y = np.full(N * N, np.nan)
    res = np.full(N * N, np.inf)
    wts = np.full((N * N, 4), np.nan)
    src = np.zeros((N * N, 4, 2), dtype=np.int64)
    for tgt, cl, s, t, Yx, Yy in cands:
        win = best[tgt] == cl
        tgt, cl, s, t, Yx, Yy = tgt[win], cl[win], s[win], t[win], Yx[win], Yy[win]
        iy, ix = cl // N, cl % N
        d_x[tgt] = (ix + s - Yx) * h
        d_y[tgt] = (iy + t - Yy) * h
        px = (p00[0].ravel()[cl] * (1 - s) * (1 - t) + p10[0].ravel()[cl] * s * (1 - t)
              + p01[0].ravel()[cl] * (1 - s) * t + p11[0].ravel()[cl] * s * t)
        py = (p00[1].ravel()[cl] * (1 - s) * (1 - t) + p10[1].ravel()[cl] * s * (1 - t)
              + p01[1].ravel()[cl] * (1 - s) * t + p11[1].ravel()[cl] * s * t)
        res[tgt] = np.maximum(np.abs(px - Yx), np.abs(py - Yy))
        wts[tgt] = np.stack([(1 - s) * (1 - t), s * (1 - t), (1 - s) * t, s * t], axis=1)
        for k, c in enumerate((c00, c10, c01, c11)):
            src[tgt, k, 0] = c[0].ravel()[cl]
            src[tgt, k, 1] = c[1].ravel()[cl]
    out = {}
    for name, f in fields.items():
        f = np.asarray(f, dtype=np.float64)
        vals = sum(wts[:, k] * f[src[:, k, 0], src[:, k, 1]] for k in range(4))
        out[name] = vals.reshape(N, N)
    return out, d_x.reshape(N, N), d_y.reshape(N, N), res.reshape(N, N)
