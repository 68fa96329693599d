"""The kinematic plane-wave driver and the alternative averaged fields on the GPU.

* LM_KINEMATIC_PLANEWAVE against the oracle's kinematic mode (same prescribed
  flow, same discretisation), element by element: 1e-12 in float64, 1e-5 in the
  mixed path.
* The exact Lagrangian means of a prescribed plane wave (section 4.2.1,
  eq. (4.8); the Adler-equation solution of oracle/closed.py) on the GPU itself,
  to the discretisation tolerances of the oracle's own pin, with second-order
  convergence of strategy 2's bilinear gathers.
* A uniform flow: xi = U s / 2 and eta = U T / 2 to roundoff.
* Potential vorticity q = (f + zeta) / h in the full dynamics without
  dissipation: material conservation (section 4.1, eq. (4.2); section 4.2.1)
  gives q~^L(x) = q(x, tau + T) for strategy 1 and q-bar^L(x) = q(x + xi(x), tau + T)
  for strategy 2.
"""

import math

import numpy as np
import pytest

from gpu_util import say
from oracle.closed import adler_frequency, omega_poincare, plane_wave_exact_means
from oracle.lagmean import Params, PlaneWave, Run as OracleRun, relative_l2
from test_oracle_pins import _grid, _smooth_flow, _trig_interp

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2208_02682_amd as L
    return L


def _wave(k=2.0, a=0.3, m=1, nsteps=400):
    """The oracle pin's plane wave along x: u amplitude a, omega from the dispersion relation."""
    omega = omega_poincare(k)
    A = k * a / omega
    Om = adler_frequency(k, a, omega)
    dt = m * 2 * math.pi / Om / nsteps
    return dict(kx=k, ky=0.0, A=A, omega=omega, phase=0.0), dt, nsteps, (k, a, omega)


def _gpu_kinematic(N, kin, dt, nsteps, fields, precision="fp64", intervals=1, pre=0):
    from paper_2208_02682_amd.lagmean import Run, make_config
    run = Run(make_config(N, precision=precision, dt=dt, fields=fields, kinematic=kin))
    if pre:
        run.step(pre)
    outs = []
    for _ in range(intervals):
        run.begin_interval()
        run.step(nsteps)
        run.end_interval()
        outs.append(run.field_outputs())
    run.close()
    return outs


def _oracle_kinematic(N, kin, dt, nsteps, fields, intervals=1, pre=0):
    waves = [PlaneWave(kin["kx"], kin["ky"], kin["A"], kin["omega"], kin.get("phase", 0.0))] if kin["A"] else []
    r = OracleRun(Params(N=N, dt=dt, fields=fields, mode="kinematic", waves=waves, U0=kin.get("U0", 0.0),
                         V0=kin.get("V0", 0.0)))
    if pre:
        r.step(pre)
    outs = []
    for _ in range(intervals):
        r.begin_interval()
        r.step(nsteps)
        outs.append(r.end_interval())
    return outs


def _rel(key, a, b, floor=1e-3):
    """Relative L2 (heights as h - H), against the larger of the reference's norm
    and an rms of `floor`: some outputs of the prescribed wave vanish exactly in
    the continuum (the mean of v, eq. (4.8) along x), and their discrete values
    are discretisation residue near 1e-8, too small to divide roundoff by."""
    if key.endswith(":h"):
        a, b = a - 1.0, b - 1.0
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), floor * np.sqrt(b.size)))


@pytest.mark.parametrize("fields", [("h", "zeta"), ("u", "v"), ("h", "q")])
def test_kinematic_plane_wave_matches_the_oracle_fp64(fields):
    kin, dt, nsteps, _ = _wave(nsteps=200)
    kin["phase"] = 0.4
    N = 64
    say(f"kinematic plane wave N={N} fields={fields} fp64")
    got = _gpu_kinematic(N, kin, dt, nsteps, fields, pre=3)[0]
    ref = _oracle_kinematic(N, kin, dt, nsteps, fields, pre=3)[0]
    assert set(got) == set(ref)
    for key in ref:
        e = _rel(key, got[key], ref[key])
        say(f"  {key}: {e:.2e}")
        assert e < 1e-12, (key, e)


def test_kinematic_oblique_wave_with_uniform_flow_matches_the_oracle():
    """A wave in a direction off the axes, with a uniform flow, over two intervals."""
    N = 64
    kin = dict(kx=-1.0, ky=2.0, A=0.04, omega=0.0, phase=1.3, U0=0.05, V0=-0.03)
    kin_o = dict(kin, omega=omega_poincare(math.sqrt(5.0)))
    dt, nsteps = 0.02, 120
    got = _gpu_kinematic(N, kin, dt, nsteps, ("h", "u"), intervals=2)
    ref = _oracle_kinematic(N, kin_o, dt, nsteps, ("h", "u"), intervals=2)
    for i in range(2):
        for key in ref[i]:
            e = _rel(key, got[i][key], ref[i][key])
            assert e < 1e-12, (i, key, e)


def test_kinematic_plane_wave_matches_the_oracle_mixed():
    kin, dt, nsteps, _ = _wave(nsteps=400)
    N = 128
    got = _gpu_kinematic(N, kin, dt, nsteps, ("h", "u"), precision="fp32")[0]
    ref = _oracle_kinematic(N, kin, dt, nsteps, ("h", "u"))[0]
    for key in ref:
        e = _rel(key, got[key], ref[key])
        say(f"  mixed {key}: {e:.2e}")
        assert e < 1e-5, (key, e)


def test_plane_wave_exact_means_on_the_gpu():
    """Every particle of the prescribed wave has the same mean velocity and depth
    (Adler equation): u_L = (omega - Omega)/k, v_L = 0, h_L = H + H k u_L / omega,
    for both strategies; the Eulerian mean of u is the plain time average."""
    errs = {}
    for N in (64, 128):
        kin, dt, nsteps, (k, a, omega) = _wave()
        uL, vL, hL = plane_wave_exact_means(k, a, omega)
        out = {}
        out.update(_gpu_kinematic(N, kin, dt, nsteps, ("u", "v"))[0])
        out.update(_gpu_kinematic(N, kin, dt, nsteps, ("h", "zeta"))[0])
        for key, ex in (("u", uL), ("v", vL), ("h", hL)):
            for S in ("S1", "S2"):
                errs[(N, S, key)] = float(np.max(np.abs(out[f"{S}_mean:{key}"] - ex)))
                say(f"  N={N} {S} mean {key}: |err| {errs[(N, S, key)]:.2e}")
        if N == 64:
            X, _ = _grid(N)
            T = nsteps * dt
            e_exact = a * (np.sin(k * X) - np.sin(k * X - omega * T)) / (omega * T)
            assert np.max(np.abs(out["E_mean:u"] - e_exact)) < 1e-9
    for key in ("u", "v", "h"):
        assert errs[(64, "S1", key)] < 1e-7        # spectral in space, RK4 in time
        assert errs[(64, "S2", key)] < 5e-4        # bilinear gathers, O(dx^2)
        assert errs[(64, "S2", key)] / max(errs[(128, "S2", key)], 1e-300) > 3.0
    assert uL > 0.02


def test_uniform_flow_displacements_are_exact_on_the_gpu():
    N, U, V, dt = 64, 0.4, -0.25, 0.03
    kin = dict(kx=0.0, ky=0.0, A=0.0, omega=0.0, phase=0.0, U0=U, V0=V)
    for prec, tol in (("fp64", 1e-13), ("fp32", 1e-6)):
        outs = _gpu_kinematic(N, kin, dt, 37, ("h", "u"), precision=prec, intervals=2, pre=5)
        T = 37 * dt
        for out in outs:
            for key, ex in (("S2_xi_x", U * T / 2), ("S2_xi_y", V * T / 2), ("S1_eta_x", U * T / 2),
                            ("S1_eta_y", V * T / 2)):
                assert np.max(np.abs(out[key] - ex)) < tol * max(1.0, abs(ex)), (prec, key)
            for S in ("S1", "S2", "E"):
                assert np.max(np.abs(out[f"{S}_mean:h"] - 1.0)) < tol
                assert np.max(np.abs(out[f"{S}_mean:u"] - U)) < tol


@pytest.mark.parametrize("interp", ["bilinear", "cubic"])
def test_gathers_wrap_displacements_beyond_one_period(interp):
    """A wave carried by a uniform drift large enough that xi = U s / 2 passes 2 pi:
    the gathers take the displaced points periodically (as the oracle's modulo),
    in both precisions."""
    from paper_2208_02682_amd.lagmean import Run, make_config
    N, dt, nsteps = 64, 0.02, 150
    kin = dict(kx=1.0, ky=0.0, A=0.05, omega=0.0, phase=0.3, U0=5.0, V0=-3.0)
    kin_o = dict(kin, omega=omega_poincare(1.0))
    out = {}
    for prec in ("fp64", "fp32"):
        run = Run(make_config(N, precision=prec, dt=dt, fields=("h", "u"), kinematic=kin, interp=interp))
        run.begin_interval()
        run.step(nsteps)
        run.end_interval()
        out[prec] = run.field_outputs()
        run.close()
    assert np.max(out["fp64"]["S2_xi_x"]) > 2 * math.pi          # displacements beyond one period
    r = OracleRun(Params(N=N, dt=dt, fields=("h", "u"), mode="kinematic", interp=interp, U0=kin["U0"],
                         V0=kin["V0"], waves=[PlaneWave(1.0, 0.0, kin["A"], kin_o["omega"], kin["phase"])]))
    r.begin_interval()
    r.step(nsteps)
    ref = r.end_interval()
    for key in ref:
        assert _rel(key, out["fp64"][key], ref[key]) < 1e-12, key
        assert _rel(key, out["fp32"][key], ref[key]) < 1e-5, key


def test_kinematic_run_has_no_state_to_set():
    L = _lib()
    from paper_2208_02682_amd.lagmean import LagMeanError, Run, make_config
    kin, dt, _, _ = _wave()
    run = Run(make_config(64, dt=dt, kinematic=kin))
    z = np.zeros((64, 64))
    with pytest.raises(LagMeanError) as e:
        run.set_state(z, z, z + 1.0)
    assert e.value.status == -2
    # the prescribed flow at time 0
    u, v, h = run.get_state()
    X, _ = _grid(64)
    a = kin["A"] * kin["omega"] / kin["kx"]
    assert np.max(np.abs(u - a * np.cos(kin["kx"] * X))) < 1e-13
    assert np.max(np.abs(h - (1.0 + kin["A"] * np.cos(kin["kx"] * X)))) < 1e-13
    run.close()
    # a wave vector outside the mask, or not an integer, is refused
    for bad in (dict(kin, kx=30.0), dict(kin, kx=1.5)):
        with pytest.raises(LagMeanError):
            Run(make_config(64, dt=dt, kinematic=bad))
    assert L is not None


def test_potential_vorticity_material_conservation_on_the_gpu():
    """q averaged along trajectories of the full dynamics (nu8 = 0): strategy 1 gives
    q(x, tau+T), strategy 2 q(x + xi, tau+T); also parity with the oracle at 1e-12."""
    from paper_2208_02682_amd.lagmean import Run, make_config
    res = {}
    for N in (64, 128):
        u, v, h = _smooth_flow(N)
        run = Run(make_config(N, dt=0.02, nu8=0.0, fields=("h", "q")))
        run.set_state(u, v, h)
        run.begin_interval()
        run.step(100)
        run.end_interval()
        out = run.field_outputs()
        uu, vv, hh = run.get_state()
        run.close()
        k = np.fft.fftfreq(N, d=1.0 / N)
        zz = np.real(np.fft.ifft2(1j * k[None, :] * np.fft.fft2(vv) - 1j * k[:, None] * np.fft.fft2(uu)))
        q = (1.0 + zz) / hh
        X, Y = _grid(N)
        res[(N, "S1")] = relative_l2(out["S1_mean:q"] - 1.0, q - 1.0)
        q_at = _trig_interp(q, X + out["S2_xi_x"], Y + out["S2_xi_y"])
        res[(N, "S2")] = relative_l2(out["S2_mean:q"] - 1.0, q_at - 1.0)
        say(f"  N={N}: S1 {res[(N, 'S1')]:.2e}, S2 {res[(N, 'S2')]:.2e}")
        if N == 64:
            o = OracleRun(Params(N=N, dt=0.02, nu8=0.0, fields=("h", "q")), u, v, h)
            o.begin_interval()
            o.step(100)
            ref = o.end_interval()
            for key in ref:
                e = _rel(key, out[key], ref[key])
                assert e < 1e-12, (key, e)
    assert res[(64, "S1")] < 1e-9
    assert res[(64, "S2")] < 3e-3
    assert res[(64, "S2")] / res[(128, "S2")] > 2.0


def test_kinematic_and_field_runs_in_a_batch_are_the_same_as_alone():
    """A kinematic run, a dynamic run averaging (u, q) and a default run advanced by
    one batch give the same bits as each alone."""
    from paper_2208_02682_amd.lagmean import Batch, Run, make_config
    kin, dt, nsteps, _ = _wave(nsteps=60)
    cfgs = [make_config(64, dt=dt, fields=("h", "u"), kinematic=kin),
            make_config(128, precision="fp32", dt=0.02, fields=("u", "q")),
            make_config(128, precision="fp32", dt=0.02)]
    states = [None, _smooth_flow(128), _smooth_flow(128)]
    steps = [nsteps, 50, 70]

    def start(cfg, st):
        r = Run(cfg)
        if st is not None:
            r.set_state(*st)
        r.begin_interval()
        return r

    alone = []
    for cfg, st, n in zip(cfgs, states, steps):
        r = start(cfg, st)
        r.step(n)
        r.end_interval()
        alone.append(r.field_outputs())
        r.close()
    runs = [start(c, st) for c, st in zip(cfgs, states)]
    with Batch() as b:
        for r, n in zip(runs, steps):
            b.add(r, n)
        while b.step(16):
            pass
        for r in runs:
            b.remove(r)
    for r, ref in zip(runs, alone):
        r.end_interval()
        got = r.field_outputs()
        r.close()
        for key in ref:
            assert np.array_equal(got[key], ref[key]), key
