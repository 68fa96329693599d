"""Launch schedules on the GPU, through the C ABI: every schedule gives the same
bits, the autotuner leaves the run it times as it was, and batches follow the
schedule table (re-capturing when it changes)."""

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu
SIZES = [(64, "fp64"), (192, "fp32"), (256, "fp64"), (384, "fp32"), (512, "fp32"), (1024, "fp32"), (1024, "fp64")]


@pytest.fixture(autouse=True)
def default_schedules():
    yield
    import paper_2208_02682_amd as L
    for n in (64, 128, 192, 256, 384, 512, 1024):
        for p in ("fp32", "fp64"):
            L.set_schedule(n, p, 0, 1)
            L.set_schedule(n, p, 0, 1, batched=True)


def _w(N, prec, seeds=(31, 32)):
    from synth.workloads import scaled_run
    return scaled_run(N, Ro=0.1, ratio=1.0, periods=1.0, seeds=seeds, precision=prec)


def _start(w, state):
    import paper_2208_02682_amd as L
    r = L.Run(L.make_config(w.N, precision=w.precision, dt=w.dt, nu8=w.nu8))
    r.set_state(*state)
    r.begin_interval()
    return r


def _finish(r):
    r.end_interval()
    out = r.outputs()
    out["xi_x_now"] = r.peek("xi_x")
    out["P_y_now"] = r.peek("P_y")
    r.close()
    return out


@pytest.mark.parametrize("N,prec", SIZES)
def test_every_schedule_gives_the_same_bits(N, prec):
    import paper_2208_02682_amd as L
    w = _w(N, prec)
    st = w.initial_state()
    steps = 6 if N < 1024 else 2
    r = _start(w, st)
    r.step(steps)
    ref = _finish(r)
    cands = L.schedule_candidates(N, prec)
    for c in cands[1:]:
        say(f"  N={N} {prec} schedule {c}")
        L.set_schedule(N, prec, *c)
        r = _start(w, st)
        r.step(steps)
        got = _finish(r)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (c, k)


def test_autotune_leaves_the_run_as_it_was():
    import paper_2208_02682_amd as L
    w = _w(256, "fp32", seeds=(41, 42))
    st = w.initial_state()
    r = _start(w, st)
    r.step(5)
    before = (r.peek("xi_x"), r.peek("u"), r.counters())
    res = r.autotune(steps=3, reps=2)
    cands = L.schedule_candidates(256, "fp32")
    say(f"  autotune 256 fp32: best {res['best']}, " + ", ".join(f"{k}: {v:.4f} ms" for k, v in res["ms"].items()))
    assert set(res["ms"]) == set(cands) and all(v > 0 for v in res["ms"].values())
    assert res["best"] == min(res["ms"], key=res["ms"].get)
    assert L.get_schedule(256, "fp32") == res["best"]
    assert np.array_equal(r.peek("xi_x"), before[0]) and np.array_equal(r.peek("u"), before[1])
    assert r.counters() == before[2] == (5, 5)
    r.step(4)
    got = _finish(r)
    L.set_schedule(256, "fp32", 0, 1)
    r = _start(w, st)
    r.step(9)
    ref = _finish(r)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k


def test_autotune_refusals():
    import paper_2208_02682_amd as L
    from paper_2208_02682_amd import LagMeanError
    r = L.Run(L.make_config(64, dt=0.01))
    with pytest.raises(LagMeanError) as e:
        r.autotune()                       # no state
    assert e.value.status == -2
    w = _w(64, "fp64")
    r.set_state(*w.initial_state())
    for steps, reps in ((0, 1), (65, 1), (4, 0), (4, 17)):
        with pytest.raises(LagMeanError) as e:
            r.autotune(steps=steps, reps=reps)
        assert e.value.status == -1
    with L.Batch() as b:
        r.begin_interval()
        b.add(r, 3)
        with pytest.raises(LagMeanError) as e:
            r.autotune()                   # inside a batch
        assert e.value.status == -2
        b.remove(r)
    r.close()


def test_batch_follows_the_schedule_table():
    import paper_2208_02682_amd as L
    specs = [(128, "fp32", 11), (192, "fp32", 9), (256, "fp64", 7)]
    ws = [_w(N, p, seeds=(50 + i, 60 + i)) for i, (N, p, _) in enumerate(specs)]
    sts = [w.initial_state() for w in ws]
    alone = []
    for w, st, (_, _, n) in zip(ws, sts, specs):
        r = _start(w, st)
        r.step(n)
        alone.append(_finish(r))
    L.set_schedule(128, "fp32", 1, 0, batched=True)
    L.set_schedule(192, "fp32", -1, 0, batched=True)
    runs = [_start(w, st) for w, st in zip(ws, sts)]
    with L.Batch() as b:
        for r, (_, _, n) in zip(runs, specs):
            b.add(r, n)
        b.step(4)
        # a change of the table between calls: the next call re-captures
        L.set_schedule(192, "fp32", 1, 1, batched=True)
        L.set_schedule(256, "fp64", -1, 0, batched=True)
        while b.step(3):
            pass
        for r in runs:
            b.remove(r)
    for i, r in enumerate(runs):
        got = _finish(r)
        for k in alone[i]:
            assert np.array_equal(got[k], alone[i][k]), (specs[i], k)


def test_batch_autotune_leaves_the_members_as_they_were():
    import paper_2208_02682_amd as L
    specs = [(128, "fp32", 10), (192, "fp32", 8), (256, "fp64", 6), (128, "fp32", 9)]
    ws = [_w(N, p, seeds=(70 + i, 80 + i)) for i, (N, p, _) in enumerate(specs)]
    sts = [w.initial_state() for w in ws]
    alone = []
    for w, st, (_, _, n) in zip(ws, sts, specs):
        r = _start(w, st)
        r.step(n)
        alone.append(_finish(r))
    runs = [_start(w, st) for w, st in zip(ws, sts)]
    with L.Batch() as b:
        for r, (_, _, n) in zip(runs, specs):
            b.add(r, n)
        b.step(3)
        before = [r.peek("xi_x") for r in runs]
        recs = b.autotune(steps=2, reps=2)
        say("  batched schedules: " + ", ".join(f"{t['n']} {t['precision']}: {t['best']}" for t in recs))
        assert sorted((t["n"], t["precision"]) for t in recs) == [(128, "fp32"), (192, "fp32"), (256, "fp64")]
        for t in recs:
            assert t["best"] in L.schedule_candidates(t["n"], t["precision"])
        for r, (_, _, n), x in zip(runs, specs, before):
            assert b.remaining(r) == n - 3
            assert r.counters() == (3, 3)
            assert np.array_equal(r.peek("xi_x"), x)
        while b.step(3):
            pass
        for r in runs:
            b.remove(r)
    for N, p, _ in specs:
        assert L.get_schedule(N, p) == (0, 1, 1)   # the single-run table is not touched
    for i, r in enumerate(runs):
        got = _finish(r)
        for k in alone[i]:
            assert np.array_equal(got[k], alone[i][k]), (specs[i], k)
