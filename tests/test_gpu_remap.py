"""Strategy-1 remap (eq. (3.8)) on the GPU against the oracle's remap of the
oracle's own strategy-1 outputs, through the C ABI."""

import numpy as np
import pytest

from gpu_util import compare_value, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu

KEYS = {"S1R_mean:h": "h", "S1R_mean:zeta": "zeta", "S1R_xi_x": "d_x", "S1R_xi_y": "d_y"}


def _oracle_remap(out, max_extent=64):
    from oracle.remap import remap_s1
    fields = {"h": out["S1_mean:h"], "zeta": out["S1_mean:zeta"]}
    rm, d_x, d_y, res = remap_s1(fields, out["S1_eta_x"], out["S1_eta_y"], max_extent=max_extent)
    rm.update(d_x=d_x, d_y=d_y)
    return rm, res


def _check(w, steps, tol, max_extent=64):
    _, ref = oracle_run(w, steps_per_interval=steps, n_intervals=1)
    run, _ = gpu_run(w, steps_per_interval=steps, n_intervals=1)
    res = run.remap_s1(max_extent)
    got = run.remap_outputs()
    run.close()
    exp, eres = _oracle_remap(ref[0], max_extent)
    for k, o in KEYS.items():
        miss = np.isnan(exp[o])
        assert np.array_equal(np.isnan(got[k]), miss), k       # the same points left uncovered
        err = compare_value(k, got[k][~miss], exp[o][~miss]) if (~miss).any() else 0.0
        say(f"  N={w.N} {w.precision} {steps} steps, max_extent {max_extent}, {k}: rel {err:.3e}"
            f" ({int(miss.sum())} uncovered)")
        assert err < tol, (k, err)
    return res, float(np.max(eres)), int(np.isnan(exp["h"]).sum())


def test_remap_of_a_whole_64_interval_matches_the_oracle():
    # within one interval eta varies by several cells per cell here (the
    # clustering of section 5): fixed-point iteration would not converge
    from synth import workload
    w = workload("sw64_fp64")
    res, eres, miss = _check(w, w.steps_per_interval, 1e-12)
    assert miss == 0 and res <= 1e-12 and eres <= 1e-12, (res, eres)


@pytest.mark.parametrize("N,prec,steps,tol", [(192, "fp64", 120, 1e-12), (128, "fp32", 200, 1e-5),
                                              (256, "fp64", 300, 1e-12)])
def test_remap_other_sizes_and_the_mixed_path(N, prec, steps, tol):
    from synth.workloads import scaled_run
    w = scaled_run(N, Ro=0.08, ratio=1.0, periods=1.0, seeds=(41, 42), precision=prec)
    res, eres, miss = _check(w, steps, tol)
    assert miss == 0 and res <= 1e-12


def test_skipped_patches_leave_the_same_points_uncovered():
    # max_extent = 1 skips every patch spanning more than one cell
    from synth import workload
    w = workload("sw64_fp64")
    res, eres, miss = _check(w, w.steps_per_interval, 1e-12, max_extent=1)
    assert miss > 0 and np.isinf(res) and np.isinf(eres)


def test_remap_rules():
    import paper_2208_02682_amd as lib
    from paper_2208_02682_amd import LagMeanError
    from synth import workload
    w = workload("sw64_fp64")
    run = lib.Run(lib.make_config(w.N, dt=w.dt, nu8=w.nu8))
    run.set_state(*w.initial_state())
    with pytest.raises(LagMeanError) as e:
        run.remap_s1()                                   # no closed interval
    assert e.value.status == -2
    run.begin_interval()
    run.step(5)
    run.end_interval()
    with pytest.raises(LagMeanError) as e:
        run.remap_outputs()                              # not remapped yet
    assert e.value.status == -2
    for bad in (0, -3, 65):
        with pytest.raises(LagMeanError) as e:
            run.remap_s1(bad)
        assert e.value.status == -1
    assert run.remap_s1() <= 1e-12
    assert set(run.remap_outputs()) == set(KEYS)
    run.begin_interval()
    run.step(3)
    run.end_interval()
    with pytest.raises(LagMeanError) as e:
        run.remap_outputs()                              # describes the previous interval
    assert e.value.status == -2
    run.close()
