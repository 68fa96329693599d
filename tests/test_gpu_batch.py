"""Batched form: uneven runs stepped together give exactly what each gives alone."""

import numpy as np
import pytest

from gpu_util import OUTPUT_KEYS, compare_value, oracle_run, say

pytestmark = pytest.mark.gpu


def _runs():
    from synth.workloads import scaled_run
    spec = [(64, "fp64", 31), (128, "fp32", 17), (192, "fp64", 23), (128, "fp32", 40), (384, "fp32", 11),
            (64, "fp32", 29), (256, "fp64", 7)]
    out = []
    for i, (N, prec, steps) in enumerate(spec):
        w = scaled_run(N, Ro=0.05 + 0.01 * i, ratio=1.0 + 0.3 * i, periods=1.0, seeds=(100 + 2 * i, 101 + 2 * i),
                       precision=prec)
        out.append((w, steps))
    return out


def _start(lib, w):
    run = lib.Run(lib.make_config(w.N, precision=w.precision, dt=w.dt, nu8=w.nu8))
    u, v, h = w.initial_state()
    run.set_state(u, v, h)
    run.begin_interval()
    return run


def test_each_run_is_the_same_alone_and_in_the_batch():
    import paper_2208_02682_amd as lib
    specs = _runs()
    alone = []
    for w, steps in specs:
        run = _start(lib, w)
        run.step(steps)
        run.end_interval()
        alone.append(run.outputs())
        run.close()
    runs = [_start(lib, w) for w, _ in specs]
    with lib.Batch() as b:
        for run, (w, steps) in zip(runs, specs):
            b.add(run, steps)
        left = b.step(10)
        assert left == sum(1 for _, steps in specs if steps > 10)
        while left:
            left = b.step(13)      # members drop out at different steps
        for run, (w, steps) in zip(runs, specs):
            assert b.remaining(run) == 0
            assert run.counters() == (steps, steps)
            b.remove(run)
    for i, (run, (w, steps)) in enumerate(zip(runs, specs)):
        run.end_interval()
        got = run.outputs()
        for k in OUTPUT_KEYS:
            assert np.array_equal(got[k], alone[i][k]), (i, w.N, w.precision, k)
        run.close()
    say(f"{len(specs)} runs identical alone and batched")


def test_batched_run_matches_the_oracle():
    import paper_2208_02682_amd as lib
    w, steps = _runs()[2]  # 192^2, float64
    _, ref = oracle_run(w, steps_per_interval=steps, n_intervals=1)
    run = _start(lib, w)
    other = _start(lib, _runs()[1][0])
    with lib.Batch() as b:
        b.add(run, steps)
        b.add(other, 5)
        while b.step(8):
            pass
        b.remove(run)
        b.remove(other)
    run.end_interval()
    got = run.outputs()
    for k in OUTPUT_KEYS:
        assert compare_value(k, got[k], ref[0][k]) < 1e-12, k
    run.close()
    other.close()


def test_batch_rules():
    import paper_2208_02682_amd as lib
    from paper_2208_02682_amd import LagMeanError
    w, _ = _runs()[0]
    run = lib.Run(lib.make_config(w.N, dt=w.dt))
    b = lib.Batch()
    u, v, h = w.initial_state()
    run.set_state(u, v, h)
    with pytest.raises(LagMeanError) as e:
        b.add(run, 3)                 # no open interval
    assert e.value.status == -2
    run.begin_interval()
    b.add(run, 3)
    with pytest.raises(LagMeanError) as e:
        b.add(run, 3)                 # already a member
    assert e.value.status == -2
    with pytest.raises(LagMeanError) as e:
        run.close()                   # cannot destroy a member
    assert e.value.status == -2
    for call in (lambda: run.step(1), run.begin_interval, run.end_interval, lambda: run.set_state(u, v, h)):
        with pytest.raises(LagMeanError) as e:
            call()                    # nor drive it through the single-run calls
        assert e.value.status == -2
    assert run.counters() == (0, 0)   # reading is allowed
    assert b.step(100) == 0
    assert run.counters() == (3, 3)
    b.close()
    run.close()


def test_many_small_members_and_a_512_member_are_the_same_alone_and_batched():
    """33 members in one batch (32 of 64^2 and 128^2, both precisions, and one of
    512^2): the run descriptors, counters and blockIdx.z indexing at scale."""
    import paper_2208_02682_amd as lib
    from synth.workloads import scaled_run
    specs = []
    for i in range(32):
        N, prec = (64, "fp64") if i % 3 == 0 else ((128, "fp32") if i % 3 == 1 else (64, "fp32"))
        w = scaled_run(N, Ro=0.03 + 0.003 * i, ratio=0.5 + 0.1 * i, periods=1.0, seeds=(500 + 2 * i, 501 + 2 * i),
                       precision=prec)
        specs.append((w, 3 + (7 * i) % 11))
    specs.append((scaled_run(512, Ro=0.1, ratio=1.0, periods=1.0, seeds=(600, 601), precision="fp32"), 9))
    alone = []
    for w, steps in specs:
        run = _start(lib, w)
        run.step(steps)
        run.end_interval()
        alone.append(run.outputs())
        run.close()
    runs = [_start(lib, w) for w, _ in specs]
    with lib.Batch() as b:
        for run, (w, steps) in zip(runs, specs):
            b.add(run, steps)
        while b.step(4):
            pass
        for run in runs:
            b.remove(run)
    for i, (run, (w, steps)) in enumerate(zip(runs, specs)):
        run.end_interval()
        got = run.outputs()
        for k in OUTPUT_KEYS:
            assert np.array_equal(got[k], alone[i][k]), (i, w.N, w.precision, k)
        run.close()
    say(f"{len(specs)} members identical alone and batched")
