"""Cubic strategy-2 gathers (LM_INTERP_CUBIC) on the GPU against the oracle with
the same option, through the C ABI."""

import numpy as np
import pytest

from gpu_util import OUTPUT_KEYS, compare_value, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu


def _parity(w, steps, tol, intervals=1):
    _, ref = oracle_run(w, steps_per_interval=steps, n_intervals=intervals, interp="cubic")
    run, got = gpu_run(w, steps_per_interval=steps, n_intervals=intervals, interp="cubic", chunk=256)
    run.close()
    for i in range(intervals):
        for k in OUTPUT_KEYS:
            err = compare_value(k, got[i][k], ref[i][k])
            say(f"  N={w.N} {w.precision} cubic, interval {i}, {k}: rel {err:.3e}")
            assert err < tol, (i, k, err)
    return got, ref


def test_cubic_whole_64_interval_matches_the_oracle():
    from synth import workload
    w = workload("sw64_fp64")
    got, ref = _parity(w, w.steps_per_interval, 1e-12)
    # the option changes strategy 2 only, and by a discretisation-sized amount
    _, lin = oracle_run(w, interp="bilinear")
    for k in ("S1_mean:h", "E_mean:zeta"):
        assert compare_value(k, ref[0][k], lin[0][k]) < 1e-14
    d = compare_value("S2_mean:zeta", ref[0]["S2_mean:zeta"], lin[0]["S2_mean:zeta"])
    assert 1e-6 < d < 0.2, d


@pytest.mark.parametrize("N,prec,steps,tol", [(192, "fp64", 60, 1e-12), (128, "fp32", 150, 1e-5),
                                              (1024, "fp32", 3, 1e-5)])
def test_cubic_other_sizes_and_the_mixed_path(N, prec, steps, tol):
    from synth.workloads import scaled_run
    w = scaled_run(N, Ro=0.08, ratio=1.0, periods=1.0, seeds=(51, 52), precision=prec)
    _parity(w, steps, tol)


def test_cubic_and_bilinear_runs_batched_together_are_the_same_as_alone():
    import paper_2208_02682_amd as lib
    from synth.workloads import scaled_run
    specs = [(128, "fp32", "cubic", 23), (128, "fp32", "bilinear", 17), (64, "fp64", "cubic", 30)]
    ws = [scaled_run(N, Ro=0.06, ratio=1.2, periods=1.0, seeds=(60 + 2 * i, 61 + 2 * i), precision=p)
          for i, (N, p, _, _) in enumerate(specs)]

    def start(w, interp):
        r = lib.Run(lib.make_config(w.N, precision=w.precision, dt=w.dt, nu8=w.nu8, interp=interp))
        r.set_state(*w.initial_state())
        r.begin_interval()
        return r

    alone = []
    for w, (_, _, interp, steps) in zip(ws, specs):
        r = start(w, interp)
        r.step(steps)
        r.end_interval()
        alone.append(r.outputs())
        r.close()
    runs = [start(w, sp[2]) for w, sp in zip(ws, specs)]
    with lib.Batch() as b:
        for r, sp in zip(runs, specs):
            b.add(r, sp[3])
        while b.step(8):
            pass
        for r in runs:
            b.remove(r)
    for i, r in enumerate(runs):
        r.end_interval()
        got = r.outputs()
        for k in OUTPUT_KEYS:
            assert np.array_equal(got[k], alone[i][k]), (i, specs[i], k)
        r.close()
