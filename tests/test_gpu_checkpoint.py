"""Checkpoint and resume in the middle of an averaging interval (lm_save / lm_restore).

A run saved after k steps of an interval and restored into a fresh run of the
same configuration (or into itself, rewound) must finish the interval with the
same outputs as the run that was never interrupted, bit for bit, in both
precisions, with the momentum 1-form and cubic gathers, and for the kinematic
driver.  Checkpoints of another configuration are refused.
"""

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _w(N, prec, seeds):
    from synth.workloads import scaled_run
    return scaled_run(N, Ro=0.08, ratio=1.0, periods=1.0, seeds=seeds, precision=prec)


CASES = [
    dict(N=256, prec="fp32", extra={}),
    dict(N=128, prec="fp64", extra=dict(momentum=True, interp="cubic")),
    dict(N=192, prec="fp32", extra=dict(fields=("u", "q"))),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c['N']}-{c['prec']}-{'-'.join(c['extra'])}")
def test_resume_mid_interval_is_bit_identical(case):
    from paper_2208_02682_amd.lagmean import Run, make_config
    w = _w(case["N"], case["prec"], (900, 901))
    cfg = make_config(w.N, precision=w.precision, dt=w.dt, nu8=w.nu8, **case["extra"])
    k1, k2 = 23, 31
    say(f"checkpoint N={w.N} {w.precision} {case['extra']}")
    ref_run = Run(cfg)
    ref_run.set_state(*w.initial_state())
    ref_run.step(5)                      # the interval does not start at step 0
    ref_run.begin_interval()
    ref_run.step(k1)
    blob = ref_run.save()
    ref_run.step(k2)
    ref_run.end_interval()
    ref = ref_run.field_outputs()
    if case["extra"].get("momentum"):
        ref.update(ref_run.momentum_outputs())
    ref_state = ref_run.get_state()

    def finish(run):
        assert run.counters() == (5 + k1 + k2, k1 + k2)
        run.end_interval()
        out = run.field_outputs()
        if case["extra"].get("momentum"):
            out.update(run.momentum_outputs())
        return out, run.get_state()

    fresh = Run(cfg)
    fresh.restore(blob)
    assert fresh.counters() == (5 + k1, k1)
    fresh.step(k2)
    for got, state in (finish(fresh),):
        for key in ref:
            assert np.array_equal(got[key], ref[key]), ("fresh", key)
        for a, b in zip(state, ref_state):
            assert np.array_equal(a, b)
    fresh.close()
    # the same run rewound to its own checkpoint
    ref_run.restore(blob)
    ref_run.step(k2)
    got, _ = finish(ref_run)
    for key in ref:
        assert np.array_equal(got[key], ref[key]), ("rewound", key)
    ref_run.close()


def test_resume_of_a_kinematic_run_and_between_intervals():
    from paper_2208_02682_amd.lagmean import Run, make_config
    kin = dict(kx=2.0, ky=-1.0, A=0.05, omega=0.0, phase=0.2, U0=0.1, V0=0.0)
    cfg = make_config(64, precision="fp64", dt=0.02, fields=("h", "u"), kinematic=kin)
    a = Run(cfg)
    a.begin_interval()
    a.step(30)
    mid = a.save()
    a.step(20)
    a.end_interval()
    ref = a.field_outputs()
    between = a.save()                   # no interval open
    a.begin_interval()
    a.step(10)
    a.end_interval()
    ref2 = a.field_outputs()
    b = Run(cfg)
    b.restore(mid)
    b.step(20)
    b.end_interval()
    got = b.field_outputs()
    for key in ref:
        assert np.array_equal(got[key], ref[key]), key
    c = Run(cfg)
    c.restore(between)
    assert c.counters() == (50, 0)
    c.begin_interval()
    c.step(10)
    c.end_interval()
    got2 = c.field_outputs()
    for key in ref2:
        assert np.array_equal(got2[key], ref2[key]), key
    for r in (a, b, c):
        r.close()


def test_checkpoints_of_other_configurations_are_refused():
    from paper_2208_02682_amd.lagmean import LagMeanError, Run, make_config
    w = _w(128, "fp32", (910, 911))
    a = Run(make_config(128, precision="fp32", dt=w.dt, nu8=w.nu8))
    a.set_state(*w.initial_state())
    a.begin_interval()
    a.step(3)
    blob = a.save()
    others = [make_config(128, precision="fp64", dt=w.dt, nu8=w.nu8),
              make_config(64, precision="fp32", dt=w.dt, nu8=w.nu8),
              make_config(128, precision="fp32", dt=w.dt * 2, nu8=w.nu8),
              make_config(128, precision="fp32", dt=w.dt, nu8=w.nu8, interp="cubic"),
              make_config(128, precision="fp32", dt=w.dt, nu8=w.nu8, fields=("h", "q"))]
    for cfg in others:
        with Run(cfg) as b:
            with pytest.raises(LagMeanError) as e:
                b.restore(blob)
            assert e.value.status == -1
    bad = blob.copy()
    bad[0] ^= 0xFF
    for blob_bad in (blob[:100], blob[:-8], bad):
        with pytest.raises(LagMeanError) as e:
            a.restore(blob_bad)
        assert e.value.status == -1
    # a refused restore leaves the run as it was
    assert a.counters() == (3, 3)
    a.close()
