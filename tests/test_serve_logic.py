"""Host logic of the served form (admission, pooling, continuous batching) with a
stand-in backend: no GPU, no library calls."""

import itertools

import pytest

from paper_2208_02682_amd.lagmean import Config
from paper_2208_02682_amd.serve import Job, Server, config_key


def cfg(n, dt=0.01):
    c = Config()
    c.n, c.precision, c.f, c.g, c.H, c.dt, c.nu8 = n, 1, 1.0, 1.0, 1.0, dt, 0.0
    c.avg_fields, c.strategies, c.interp, c.mode = 3, 7, 0, 0
    return c


class FakeRun:
    ids = itertools.count()

    def __init__(self, c):
        self.n = c.n
        self.id = next(self.ids)
        self.steps = 0
        self.member = False
        self.budget = 0
        self.alive = True


class FakeBackend:
    """Runs as step counters; a member takes min(n, its budget) steps per call,
    as lm_batch_step does."""

    def __init__(self):
        self.created, self.destroyed, self.log = [], [], []

    def footprint(self, c):
        return c.n * c.n * 100

    def create(self, c):
        r = FakeRun(c)
        self.created.append(r)
        return r

    def start(self, run, job):
        assert run.alive and not run.member and job.state is not None
        run.steps, run.member, run.budget = 0, True, job.steps
        self.log.append(("start", job.id, run.id))

    def step(self, n):
        assert n >= 1
        for r in self.created:
            if r.alive and r.member:
                k = min(n, r.budget)
                r.steps += k
                r.budget -= k

    def finish(self, run, keep):
        assert run.member and run.budget == 0
        run.member = False
        self.log.append(("finish", run.id))
        return run.steps * 0.01, ({"steps": run.steps, "run": run.id} if keep else None)

    def abandon(self, run):
        run.member = False

    def destroy(self, run):
        assert not run.member
        run.alive = False
        self.destroyed.append(run)

    def close(self):
        pass


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1.0
        return self.t


def drain(s, limit=10000):
    done = []
    for _ in range(limit):
        if not s.busy():
            return done
        done += s.tick()
    raise AssertionError("server did not drain")


def job(i, n, steps, t=0.0):
    return Job(i, cfg(n), state=("u", "v", "h"), steps=steps, arrival=t)


def test_every_request_gets_exactly_its_steps_and_its_means():
    be = FakeBackend()
    s = Server(10**9, tick_steps=7, backend=be, clock=Clock())
    steps = [5, 13, 1, 40, 7, 22, 9]
    for i, k in enumerate(steps):
        s.submit(job(i, 64 if i % 2 else 128, k))
    done = drain(s)
    assert sorted(j.id for j in done) == list(range(len(steps)))
    for j in done:
        assert j.error is None
        assert j.outputs["steps"] == steps[j.id]
        assert j.T == pytest.approx(steps[j.id] * 0.01)
        assert j.arrival <= j.admitted <= j.finished
        assert j.state is None  # the host copy is released once uploaded


def test_admission_respects_the_budget_in_arrival_order():
    be = FakeBackend()
    fp = 128 * 128 * 100
    s = Server(2 * fp, tick_steps=100, backend=be, clock=Clock())
    for i, k in enumerate([10, 20, 5, 5]):
        s.submit(job(i, 128, k))
    done = s.tick()
    assert len(s.active) <= 2 and s.used <= 2 * fp
    done += drain(s)
    starts = [e[1] for e in be.log if e[0] == "start"]
    assert starts == [0, 1, 2, 3]                      # first come, first served
    assert len(be.created) == 2                        # never more than the budget holds
    assert {j.id for j in done} == {0, 1, 2, 3}


def test_finished_runs_are_reused_by_the_same_configuration():
    be = FakeBackend()
    s = Server(10**9, tick_steps=4, backend=be, clock=Clock())
    for i in range(6):
        s.submit(job(i, 64, 3))
        drain(s)
    assert len(be.created) == 1 and s.created == 1


def test_idle_runs_of_other_configurations_are_released_when_room_is_needed():
    be = FakeBackend()
    s = Server(256 * 256 * 100, tick_steps=4, backend=be, clock=Clock())
    s.submit(job(0, 128, 3))
    drain(s)
    s.submit(job(1, 256, 3))                           # needs the whole budget
    done = drain(s)
    assert done[0].error is None and s.evicted == 1
    assert be.destroyed and be.destroyed[0].n == 128
    assert s.used == 256 * 256 * 100


def test_resident_point_cap_queues_instead_of_widening_the_batch():
    be = FakeBackend()
    s = Server(10**9, max_resident_points=2 * 64 * 64, tick_steps=1, backend=be, clock=Clock())
    for i in range(5):
        s.submit(job(i, 64, 3))
    peak = 0
    while s.busy():
        s.tick()
        peak = max(peak, s.resident_points)
    assert peak == 2 * 64 * 64


def test_a_request_that_can_never_fit_is_rejected_not_stuck():
    be = FakeBackend()
    s = Server(64 * 64 * 100, backend=be, clock=Clock())
    s.submit(job(0, 128, 3))
    s.submit(job(1, 64, 3))
    done = drain(s)
    by = {j.id: j for j in done}
    assert by[0].error and by[0].outputs is None
    assert by[1].error is None and by[1].outputs["steps"] == 3


def test_tick_never_passes_the_earliest_finishing_run():
    be = FakeBackend()
    s = Server(10**9, tick_steps=50, backend=be, clock=Clock())
    s.submit(job(0, 64, 3))
    s.submit(job(1, 64, 100))
    first = s.tick()
    assert [j.id for j in first] == [0]                # retired after exactly 3 steps
    assert s.active[0][2] == 97
    with pytest.raises(ValueError):
        s.submit(job(2, 64, 0))


def test_config_key_separates_precision_and_size():
    a, b, c = cfg(64), cfg(64), cfg(128)
    b.precision = 0
    assert config_key(a) != config_key(b) and config_key(a) != config_key(c)
    assert config_key(a) == config_key(cfg(64))
