"""lm_batch_step_static (the allocation-free batched step) against lm_batch_step.

Both advance the same runs from the same states with the same kernels; the
outputs must agree bit for bit.  Two static calls in a row, the second with a
smaller batch (fewer and smaller runs), check that what the first left in the
shared device scratch does not leak into the second.  A batch above the member
limit is refused before anything is launched.
"""

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _state(N, seed):
    from synth.workloads import scaled_run
    return scaled_run(N, Ro=0.1, ratio=1.0, periods=1.0, seeds=(seed, seed + 1)).initial_state()


def _make(cfgs, states):
    from paper_2208_02682_amd.lagmean import Run
    runs = []
    for cfg, st in zip(cfgs, states):
        r = Run(cfg)
        r.set_state(*st)
        r.begin_interval()
        runs.append(r)
    return runs


def _batched(cfgs, states, steps, static, tick):
    """Outputs of the runs advanced in one batch by lm_batch_step or lm_batch_step_static."""
    from paper_2208_02682_amd.lagmean import Batch
    runs = _make(cfgs, states)
    with Batch() as b:
        for r, n in zip(runs, steps):
            b.add(r, n)
        while (b.step_static(tick) if static else b.step(tick)):
            pass
        for r in runs:
            b.remove(r)
    outs = []
    for r in runs:
        r.end_interval()
        outs.append(r.field_outputs())
        r.close()
    return outs


def _check_same(cfgs, states, steps, tick):
    ref = _batched(cfgs, states, steps, static=False, tick=tick)
    got = _batched(cfgs, states, steps, static=True, tick=tick)
    for i, (a, b) in enumerate(zip(got, ref)):
        for key in b:
            assert np.array_equal(a[key], b[key]), (i, cfgs[i].n, key)


def test_static_step_equals_the_graph_step_on_two_calls_in_a_row():
    from paper_2208_02682_amd.lagmean import make_config
    # first call: five runs of three sizes, both precisions, a cubic-gather run
    # and one averaging other fields; members drop out at different steps
    big = [make_config(256, precision="fp32", dt=0.0025),
           make_config(192, precision="fp32", dt=0.0033, interp="cubic"),
           make_config(128, precision="fp64", dt=0.005),
           make_config(128, precision="fp32", dt=0.005, fields=("u", "q")),
           make_config(256, precision="fp32", dt=0.0025)]
    big_states = [_state(256, 11), _state(192, 13), _state(128, 15), _state(128, 17), _state(256, 19)]
    say("static step: first call, 5 runs (N 128..256)")
    _check_same(big, big_states, [40, 33, 27, 35, 21], tick=16)
    # second call: a smaller batch (two 64^2 runs)
    small = [make_config(64, precision="fp64", dt=0.01), make_config(64, precision="fp32", dt=0.01)]
    say("static step: second call, 2 runs (N 64)")
    _check_same(small, [_state(64, 21), _state(64, 23)], [19, 25], tick=8)


def test_static_step_refuses_a_batch_above_its_limit():
    from paper_2208_02682_amd.lagmean import Batch, LagMeanError, LM_STATIC_MAX_MEMBERS, make_config
    cfg = make_config(64, precision="fp64", dt=0.01)
    st = _state(64, 31)
    runs = _make([cfg] * (LM_STATIC_MAX_MEMBERS + 1), [st] * (LM_STATIC_MAX_MEMBERS + 1))
    try:
        with Batch() as b:
            for r in runs:
                b.add(r, 3)
            with pytest.raises(LagMeanError) as e:
                b.step_static(1)
            assert e.value.status == -7 and "LM_STATIC_MAX_MEMBERS" in str(e.value)
            # nothing was launched: every member still has its whole budget
            assert all(b.remaining(r) == 3 for r in runs)
            assert all(r.counters()[1] == 0 for r in runs)
            for r in runs:
                b.remove(r)
    finally:
        for r in runs:
            r.close()
