"""Pins of the oracle's strategy-1 remap (eq. (3.8)) against what the mathematics
fixes: exact shifts, an explicit bilinear formula, smooth lift maps known in
closed form (inverted by Newton's method), mild and strongly sheared, and
agreement with strategy 2 on the same particles."""

import numpy as np

from oracle.remap import remap_s1
from test_oracle_pins import _grid, _tracked_case


def test_whole_cell_offset_is_an_exact_shift():
    N = 32
    dx = 2 * np.pi / N
    rng = np.random.default_rng(3)
    f = rng.standard_normal((N, N))
    eta_x = np.full((N, N), 2 * dx)
    eta_y = np.full((N, N), -3 * dx)
    out, d_x, d_y, res = remap_s1({"f": f}, eta_x, eta_y)
    # f-bar(y) = f~(y + eta): element (iy, ix) takes f[iy - 3, ix + 2]
    assert np.array_equal(out["f"], np.roll(np.roll(f, -2, axis=1), 3, axis=0))
    assert np.allclose(d_x, 2 * dx, rtol=0, atol=1e-15) and np.allclose(d_y, -3 * dx, rtol=0, atol=1e-15)
    assert np.max(res) <= 1e-12


def test_constant_fractional_offset_matches_explicit_bilinear_weights():
    N = 24
    dx = 2 * np.pi / N
    rng = np.random.default_rng(4)
    f = rng.standard_normal((N, N))
    ox, oy = 1.37, -0.61  # cells
    out, d_x, d_y, _ = remap_s1({"f": f}, np.full((N, N), ox * dx), np.full((N, N), oy * dx))
    # corners (iy + fy + {0,1}, ix + fx + {0,1}) with weights from the fractional parts
    fx, fy = int(np.floor(ox)), int(np.floor(oy))
    ax, ay = ox - fx, oy - fy
    s = lambda a, b: np.roll(np.roll(f, -a, axis=1), -b, axis=0)
    ref = ((1 - ax) * (1 - ay) * s(fx, fy) + ax * (1 - ay) * s(fx + 1, fy)
           + (1 - ax) * ay * s(fx, fy + 1) + ax * ay * s(fx + 1, fy + 1))
    assert np.max(np.abs(out["f"] - ref)) < 1e-14
    assert np.allclose(d_x, ox * dx, rtol=0, atol=1e-14) and np.allclose(d_y, oy * dx, rtol=0, atol=1e-14)


def _lift(YX, YY, a=0.25, b=0.2):
    """A smooth invertible lift map Xi(y) = y + A(y) and the Jacobian of A."""
    Ax = a * np.sin(YY + 0.3) + 0.1 * np.sin(YX)
    Ay = b * np.cos(YX - 0.7)
    J = (0.1 * np.cos(YX), a * np.cos(YY + 0.3), -b * np.sin(YX - 0.7), np.zeros_like(YX))
    return Ax, Ay, J


def _mean_field(YX, YY):
    return np.cos(YX) * np.sin(2 * YY) + 0.5 * np.sin(YX + YY)


def _inverse_lift(N, a=0.25, b=0.2):
    """Grid, and Xi^{-1}(x) by damped Newton on y + A(y) = x, to roundoff."""
    X, Y = _grid(N)
    yx, yy = X.copy(), Y.copy()
    for it in range(200):
        Ax, Ay, (j11, j12, j21, j22) = _lift(yx, yy, a, b)
        rx, ry = yx + Ax - X, yy + Ay - Y
        a11, a12, a21, a22 = 1 + j11, j12, j21, 1 + j22
        det = a11 * a22 - a12 * a21
        lam = 0.5 if it < 20 else 1.0
        yx = yx - lam * (a22 * rx - a12 * ry) / det
        yy = yy - lam * (-a21 * rx + a11 * ry) / det
    assert max(np.max(np.abs(rx)), np.max(np.abs(ry))) < 1e-13 and np.min(det) > 0.1
    return X, Y, yx, yy


def _remap_error(N, a=0.25, b=0.2):
    X, Y, yx, yy = _inverse_lift(N, a, b)
    eta_x, eta_y = X - yx, Y - yy          # x - Xi^{-1}(x)
    ftil = _mean_field(yx, yy)             # f~(x) = f-bar(Xi^{-1}(x)), eq. (3.8)
    out, d_x, d_y, res = remap_s1({"f": ftil}, eta_x, eta_y)
    assert np.max(res) <= 1e-12
    Ax, Ay, _ = _lift(X, Y, a, b)
    return (np.max(np.abs(out["f"] - _mean_field(X, Y))),
            max(np.max(np.abs(d_x - Ax)), np.max(np.abs(d_y - Ay))))


def test_smooth_lift_map_is_recovered_at_second_order():
    e = {N: _remap_error(N) for N in (32, 64, 128)}
    for k in (0, 1):
        assert e[128][k] < 0.02
        # bilinear interpolation: O(dx^2), ratio ~4 per doubling
        assert 3.0 < e[32][k] / e[64][k] < 5.0 and 3.0 < e[64][k] / e[128][k] < 5.0, e


def test_strongly_sheared_lift_map_beyond_fixed_point_iteration():
    # eta varies by several cells per cell: the plain iteration x <- y + eta(x)
    # does not converge, the patch inversion still recovers the map and the mean
    from oracle.lagmean import bilinear_periodic
    a, b = 1.5, 0.5
    N = 64
    X, Y, yx, yy = _inverse_lift(N, a, b)
    h = 2 * np.pi / N
    eta_x, eta_y = X - yx, Y - yy
    assert np.max(np.abs(np.diff(eta_x / h, axis=0))) > 5.0
    d_x, d_y = eta_x.copy(), eta_y.copy()
    for _ in range(200):
        n_x, n_y = bilinear_periodic(eta_x, d_x, d_y, h), bilinear_periodic(eta_y, d_x, d_y, h)
        step = np.maximum(np.abs(n_x - d_x), np.abs(n_y - d_y)) / h
        d_x, d_y = n_x, n_y
    assert np.max(step) > 1e-3
    e = {N: _remap_error(N, a, b) for N in (64, 128, 256)}
    for k in (0, 1):
        assert e[64][k] > e[128][k] > e[256][k] and e[128][k] / e[256][k] > 3.3, e
        assert e[256][k] < 0.01, e


def test_remapped_strategy1_matches_strategy2_on_the_same_particles():
    # the remap turns strategy 1 into strategy 2's variables: xi(y) and f-bar(y)
    N = 32
    out, _ = _tracked_case(N)
    fields = {k: out[f"S1_mean:{k}"] for k in ("h", "u")}
    rm, d_x, d_y, res = remap_s1(fields, out["S1_eta_x"], out["S1_eta_y"])
    assert np.max(res) <= 1e-12
    for a, b in ((d_x, out["S2_xi_x"]), (d_y, out["S2_xi_y"]), (rm["h"], out["S2_mean:h"]), (rm["u"], out["S2_mean:u"])):
        err = np.max(np.abs(a - b))
        assert err < 2e-3
        assert err < 0.05 * np.max(np.abs(b - b.mean()))


def test_where_the_mean_map_folds_the_lowest_cell_index_decides():
    """A closed-form fold: eta_x = 8 cells sin(2 pi x / N), eta_y = 0, so the mean
    map x -> x - eta(x) (piecewise linear between grid values along x) is not
    monotone near x = 0 and x - eta(x) = y has three roots for some grid points y.
    Every root is a particle whose mean position is y (the paper's caveat about
    clustering mean positions, section 5): any covering patch solves eq. (3.8).
    The stated rule takes the patch of the lowest cell index iy N + ix.  Here every
    covering segment of every row is enumerated directly and solved in closed
    form, and the oracle must return the root of the lowest covering cell; the
    test field takes different values at the different roots, so another choice
    fails."""
    N = 32
    h = 2 * np.pi / N
    i = np.arange(N)
    amp = 8.0                                            # cells; amp * 2 pi / N > 1 folds the map
    e1 = amp * np.sin(2 * np.pi * i / N)                 # eta_x in cells along x
    eta_x = np.broadcast_to(e1[None, :] * h, (N, N)).copy()
    eta_y = np.zeros((N, N))
    X, Y = _grid(N)
    ftil = np.cos(X) + 0.4 * np.sin(X / 1.0 + 0.3) + 0.3 * np.sin(2 * Y)
    out, d_x, d_y, res = remap_s1({"f": ftil}, eta_x, eta_y)
    m = np.arange(N + 1) - np.append(e1, e1[0])          # x - eta(x) at x = 0..N (cells, unwrapped)
    multi = 0
    for iy in range(N):
        # a grid point on row iy is covered by cells of rows iy - 1 (t = 1) and iy
        # (t = 0); eta does not depend on y, so both rows give the same roots in x
        # and the lowest cell index is the lowest covering ix
        for yx in range(N):
            roots = []
            for ix in range(N):
                a, b = m[ix], m[ix + 1]
                for k in (-1, 0, 1):
                    yk = yx + k * N
                    if min(a, b) - 1e-12 <= yk <= max(a, b) + 1e-12 and a != b:
                        s = (yk - a) / (b - a)
                        roots.append((ix, ix + s, yk))
            assert roots, (iy, yx)
            distinct = {round(x, 9) for _, x, _ in roots}
            if len(distinct) > 1:
                multi += 1
            ix, x, yk = min(roots)                          # the lowest covering cell of the row
            assert abs(d_x[iy, yx] - (x - yk) * h) < 1e-12, (iy, yx, roots)
            assert abs(d_y[iy, yx]) < 1e-12
            # f~ at the root: linear along x between the grid values of the row
            j0 = int(np.floor(x)) % N
            frac = x - np.floor(x)
            want = (1 - frac) * ftil[iy, j0] + frac * ftil[iy, (j0 + 1) % N]
            assert abs(out["f"][iy, yx] - want) < 1e-12, (iy, yx)
    assert multi >= 3 * N                                  # the rule decided on many points
    assert np.max(res) <= 1e-12
