"""Parity of the HIP path with the CPU FP64 oracle (element by element, same seeded inputs).

Tolerances (relative L2 over the grid, heights as h - H, positions as
displacements): 1e-12 for the float64 path, 1e-5 for the mixed path (float32
transforms, float64 displacement/position state).
"""

import math

import numpy as np
import pytest

from gpu_util import OUTPUT_KEYS, compare_value, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def lib():
    import paper_2208_02682_amd as p
    return p


def _band_limited(N, seed, K=None):
    """Random real fields whose spectra lie inside the 2/3-rule mask."""
    rng = np.random.default_rng(seed)
    K = K if K is not None else (N - 1) // 3
    out = []
    for _ in range(3):
        a = rng.standard_normal((N, N))
        A = np.fft.rfft2(a)
        ky = np.fft.fftfreq(N, d=1.0 / N)[:, None]
        kx = np.arange(N // 2 + 1)[None, :]
        A *= (np.abs(kx) <= K) & (np.abs(ky) <= K)
        out.append(np.fft.irfft2(A, s=(N, N)))
    return out


@pytest.mark.parametrize("N", [64, 128, 192, 256, 384, 512, 1024])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_set_get_state_roundtrip(lib, N, prec):
    say(f"roundtrip N={N} {prec}")
    u, v, h = _band_limited(N, 1)
    h = h + 1.0
    run = lib.Run(lib.make_config(N, precision=prec, dt=0.01))
    run.set_state(u, v, h)
    uu, vv, hh = run.get_state()
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert np.max(np.abs(uu - u)) < tol * np.max(np.abs(u))
    assert np.max(np.abs(vv - v)) < tol * np.max(np.abs(v))
    assert np.max(np.abs(hh - h)) < tol * np.max(np.abs(h))
    # components outside the mask are removed
    w = np.random.default_rng(3).standard_normal((N, N))
    run.set_state(w, w, 1.0 + w)
    uu, _, _ = run.get_state()
    W = np.fft.rfft2(w)
    K = (N - 1) // 3
    ky = np.fft.fftfreq(N, d=1.0 / N)[:, None]
    kx = np.arange(N // 2 + 1)[None, :]
    wm = np.fft.irfft2(W * ((kx <= K) & (np.abs(ky) <= K)), s=(N, N))
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert np.max(np.abs(uu - wm)) < tol
    run.close()


def _oracle_fields(r):
    keys = {"u": "u", "v": "v", "h": "h", "gbar:h": "gbar:h", "gbar:zeta": "gbar:zeta",
            "gtil:h": "gtil:h", "gtil:zeta": "gtil:zeta", "E:h": "E:h", "E:zeta": "E:zeta",
            "xi_x": "xi_x", "xi_y": "xi_y", "P_x": "P_x", "P_y": "P_y"}
    return {k: r.physical(v) for k, v in keys.items()}


@pytest.mark.parametrize("nsteps", [1, 3])
def test_first_steps_every_field_fp64(lib, nsteps):
    """Each of the 13 prognostic fields after a few steps (the interval starts at
    step 0, so stage 1 of step 1 exercises the t = tau limit)."""
    from synth import workload
    from oracle.lagmean import Params, Run as ORun
    w = workload("sw64_fp64")
    u, v, h = w.initial_state()
    say(f"first steps N=64 nsteps={nsteps}")
    o = ORun(Params(N=64, dt=w.dt, nu8=w.nu8), u, v, h)
    o.begin_interval()
    o.step(nsteps)
    ref = _oracle_fields(o)
    run = lib.Run(lib.make_config(64, precision="fp64", dt=w.dt, nu8=w.nu8))
    run.set_state(u, v, h)
    run.begin_interval()
    run.step(nsteps)
    for k, b in ref.items():
        a = run.peek(k)
        err = compare_value(k, a, b)
        say(f"  {k}: rel {err:.3e}")
        assert err < TOL64, k
    run.close()


def test_full_interval_sw64_fp64(lib):
    """64^2 FP64 single run: one whole averaging interval (1012 steps), all outputs."""
    from synth import workload
    w = workload("sw64_fp64")
    say("oracle sw64 ...")
    _, ref = oracle_run(w)
    say("gpu sw64 ...")
    run, got = gpu_run(w, chunk=256)
    for k in OUTPUT_KEYS:
        err = compare_value(k, got[0][k], ref[0][k])
        say(f"  {k}: rel {err:.3e}")
        assert err < TOL64, k
    # the means differ from the Eulerian ones: the comparison is not vacuous
    assert compare_value("h", ref[0]["S2_mean:h"], ref[0]["E_mean:h"]) > 1e-3
    run.close()


def test_two_intervals_short_sw64_fp64(lib):
    """Successive intervals: the second restarts the means while the flow goes on."""
    from synth import workload
    w = workload("sw64_fp64")
    _, ref = oracle_run(w, steps_per_interval=37, n_intervals=2)
    run, got = gpu_run(w, steps_per_interval=37, n_intervals=2)
    for i in range(2):
        for k in OUTPUT_KEYS:
            err = compare_value(k, got[i][k], ref[i][k])
            assert err < TOL64, (i, k, err)
    run.close()


@pytest.mark.parametrize("name,steps", [("sw256_fp64", 12)])
def test_short_run_full_size_fp64(lib, name, steps):
    from synth import workload
    w = workload(name)
    say(f"{name}: {steps} steps")
    _, ref = oracle_run(w, steps_per_interval=steps, n_intervals=1)
    run, got = gpu_run(w, steps_per_interval=steps, n_intervals=1)
    for k in OUTPUT_KEYS:
        err = compare_value(k, got[0][k], ref[0][k])
        say(f"  {k}: rel {err:.3e}")
        assert err < TOL64, k
    run.close()


@pytest.mark.parametrize("N,prec", [(128, "fp64"), (192, "fp64"), (384, "fp64"), (192, "fp32"), (512, "fp32")])
def test_short_run_every_grid_size(lib, N, prec):
    """Every supported N (radix-2 and radix-3 transforms) against the oracle."""
    from synth.workloads import scaled_run
    w = scaled_run(N, Ro=0.08, ratio=1.5, periods=1.0, seeds=(31, 32), precision=prec)
    steps = 9
    say(f"N={N} {prec}: {steps} steps")
    _, ref = oracle_run(w, steps_per_interval=steps, n_intervals=1)
    run, got = gpu_run(w, steps_per_interval=steps, n_intervals=1)
    tol = TOL64 if prec == "fp64" else TOL32
    for k in OUTPUT_KEYS:
        err = compare_value(k, got[0][k], ref[0][k])
        say(f"  {k}: rel {err:.3e}")
        assert err < tol, k
    run.close()


def test_short_run_1024_fp32(lib):
    """1024^2 mixed path against the FP64 oracle over a few steps, all outputs."""
    from synth import workload
    w = workload("sw1024_fp32")
    steps = 3
    say("oracle 1024 ...")
    _, ref = oracle_run(w, steps_per_interval=steps, n_intervals=1)
    say("gpu 1024 fp32 ...")
    run, got = gpu_run(w, steps_per_interval=steps, n_intervals=1)
    for k in OUTPUT_KEYS:
        err = compare_value(k, got[0][k], ref[0][k])
        say(f"  {k}: rel {err:.3e}")
        assert err < TOL32, k
    run.close()


def test_full_interval_sw64_fp32(lib):
    """Mixed path over a whole 64^2 interval against the FP64 oracle."""
    from synth import workload
    w = workload("sw64_fp64").with_(precision="fp32")
    _, ref = oracle_run(w)
    run, got = gpu_run(w, chunk=256)
    errs = {k: compare_value(k, got[0][k], ref[0][k]) for k in OUTPUT_KEYS}
    for k in OUTPUT_KEYS:
        say(f"  {k}: rel {errs[k]:.3e}")
    for k in OUTPUT_KEYS:
        assert errs[k] < TOL32, k
    run.close()


def test_error_paths(lib):
    from paper_2208_02682_amd import LagMeanError
    run = lib.Run(lib.make_config(64, dt=0.01))
    with pytest.raises(LagMeanError) as e:
        run.begin_interval()
    assert e.value.status == -2
    u = np.zeros((64, 64))
    run.set_state(u, u, u + 1.0)
    with pytest.raises(LagMeanError) as e:
        run.end_interval()
    assert e.value.status == -2
    run.begin_interval()
    with pytest.raises(LagMeanError) as e:
        run.end_interval()   # no step
    assert e.value.status == -2
    with pytest.raises(LagMeanError):
        run.read_mean(0, 0)
    with pytest.raises(LagMeanError) as e:
        run.step(-1)
    assert e.value.status == -1
    run.step(2)
    T = run.end_interval()
    assert abs(T - 0.02) < 1e-15
    # a NaN in the input reaches the outputs and is reported
    bad = u.copy()
    bad[3, 5] = np.nan
    run.set_state(bad, u, u + 1.0)
    run.begin_interval()
    run.step(1)
    with pytest.raises(LagMeanError) as e:
        run.end_interval()
    assert e.value.status == -5
    run.close()
