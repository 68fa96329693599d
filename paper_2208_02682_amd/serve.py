"""Served form: averaging requests admitted by HBM footprint and advanced by
continuous batching.

A request is one averaging interval of one run: an initial state (u, v, h),
a configuration and a number of RK4 steps; its answer is the interval's means
(strategy 1, strategy 2 and Eulerian, the outputs of ``Run.outputs``).  The
server keeps every admitted run resident in device memory and advances all of
them together through one ``lm_batch``: a tick advances every resident run by
the same number of steps (at most ``tick_steps``, and never past the earliest
finishing run), then retires the finished runs, then admits queued requests.

Admission is first come, first served.  A request is admitted when
  * the runs already created plus its own footprint (``lm_query_footprint``)
    fit in ``hbm_budget`` bytes, after releasing idle runs of other
    configurations if needed, and
  * the resident grid points stay within ``max_resident_points`` (when set), so
    that a tick stays short and queued requests wait in order instead of
    slowing every resident run down.
Finished runs go back to a pool keyed by configuration and are reused by the
next request of the same configuration (no device allocation on that path).

The scheduling logic talks to a small backend interface so that it can be
exercised without a GPU; ``HipBackend`` is the real one.
"""

from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

from .lagmean import Batch, Config, Run, footprint


def config_key(cfg: Config) -> tuple:
    """Runs with equal keys are interchangeable (same buffers and constants)."""
    return (cfg.n, cfg.precision, cfg.f, cfg.g, cfg.H, cfg.dt, cfg.nu8, cfg.avg_fields, cfg.strategies,
            cfg.interp, cfg.mode)


@dataclass
class Job:
    """One averaging request.  ``arrival`` is on the server's clock."""
    id: Any
    cfg: Config
    state: Optional[tuple]          # (u, v, h), released once uploaded
    steps: int
    arrival: float
    admitted: Optional[float] = None
    finished: Optional[float] = None
    T: Optional[float] = None
    outputs: Optional[Dict[str, Any]] = field(default=None, repr=False)
    error: Optional[str] = None

    @property
    def points(self) -> int:
        return int(self.cfg.n) * int(self.cfg.n)

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class HipBackend:
    """Runs and one batch of the HIP library, all on one stream."""

    def __init__(self, stream: int = 0):
        self.stream = stream
        self.batch = Batch(stream)

    def footprint(self, cfg: Config) -> int:
        return footprint(cfg)

    def create(self, cfg: Config) -> Run:
        return Run(cfg, stream=self.stream)

    def start(self, run: Run, job: Job) -> None:
        run.set_state(*job.state)
        run.begin_interval()
        self.batch.add(run, job.steps)

    def step(self, nsteps: int) -> None:
        self.batch.step(nsteps)

    def remaining(self, run: Run) -> int:
        return self.batch.remaining(run)

    def finish(self, run: Run, keep_outputs: bool):
        self.batch.remove(run)
        T = run.end_interval()
        return T, (run.outputs() if keep_outputs else None)

    def abandon(self, run: Run) -> None:
        if run in self.batch.members:
            self.batch.remove(run)

    def destroy(self, run: Run) -> None:
        run.close()

    def close(self) -> None:
        self.batch.close()


class Server:
    def __init__(self, hbm_budget: int, *, max_resident_points: Optional[int] = None, tick_steps: int = 32,
                 keep_outputs: bool = True, backend=None, clock: Callable[[], float] = time.perf_counter):
        if tick_steps < 1:
            raise ValueError("tick_steps must be >= 1")
        self.budget = int(hbm_budget)
        self.max_points = max_resident_points
        self.tick_steps = int(tick_steps)
        self.keep_outputs = keep_outputs
        self.backend = backend if backend is not None else HipBackend()
        self.clock = clock
        self.queue: collections.deque = collections.deque()
        self.active: List[list] = []      # [job, run, remaining steps]
        self.idle: Dict[tuple, List[Any]] = collections.OrderedDict()
        self.sizes: Dict[int, int] = {}   # id(run) -> footprint of every created run
        self.used = 0
        self.created = 0
        self.evicted = 0
        self.rejected: List[Job] = []

    # -- bookkeeping -------------------------------------------------------
    @property
    def resident_points(self) -> int:
        return sum(j.points for j, _, _ in self.active)

    def busy(self) -> bool:
        return bool(self.queue or self.active)

    def submit(self, job: Job) -> None:
        if job.steps < 1:
            raise ValueError("a request needs at least one step")
        self.queue.append(job)

    # -- admission ---------------------------------------------------------
    def _acquire(self, cfg: Config):
        key = config_key(cfg)
        pool = self.idle.get(key)
        if pool:
            run = pool.pop()
            if not pool:
                del self.idle[key]
            return run
        need = self.backend.footprint(cfg)
        # release idle runs of other configurations, least recently used first
        while self.used + need > self.budget and self.idle:
            k = next(iter(self.idle))
            victim = self.idle[k].pop(0)
            if not self.idle[k]:
                del self.idle[k]
            self.backend.destroy(victim)
            self.used -= self.sizes.pop(id(victim))
            self.evicted += 1
        if self.used + need > self.budget:
            return None
        run = self.backend.create(cfg)
        self.sizes[id(run)] = need
        self.used += need
        self.created += 1
        return run

    def _release(self, run, cfg: Config) -> None:
        key = config_key(cfg)
        self.idle.setdefault(key, []).append(run)
        self.idle.move_to_end(key)

    def _admit(self) -> None:
        while self.queue:
            job = self.queue[0]
            if self.backend.footprint(job.cfg) > self.budget:
                self.queue.popleft()
                job.error = "footprint exceeds the HBM budget"
                self.rejected.append(job)
                continue
            if self.max_points is not None and self.active and \
                    self.resident_points + job.points > self.max_points:
                return
            run = self._acquire(job.cfg)
            if run is None:
                return
            self.queue.popleft()
            try:
                self.backend.start(run, job)
            except Exception as e:  # the run may hold a partial state: drop it
                job.error = str(e)
                self.rejected.append(job)
                self.backend.abandon(run)
                self.backend.destroy(run)
                self.used -= self.sizes.pop(id(run))
                continue
            job.state = None
            job.admitted = self.clock()
            self.active.append([job, run, job.steps])

    # -- one tick ----------------------------------------------------------
    def tick(self) -> List[Job]:
        """Admit, advance every resident run, retire the finished ones.
        Returns the jobs finished (or failed) in this tick."""
        out: List[Job] = []
        self._admit()
        if self.rejected:
            out.extend(self.rejected)
            self.rejected = []
        if not self.active:
            return out
        n = min(self.tick_steps, min(a[2] for a in self.active))
        self.backend.step(n)
        still = []
        for a in self.active:
            a[2] -= n
            if a[2] > 0:
                still.append(a)
                continue
            job, run, _ = a
            try:
                job.T, job.outputs = self.backend.finish(run, self.keep_outputs)
            except Exception as e:
                job.error = str(e)
            job.finished = self.clock()
            self._release(run, job.cfg)
            out.append(job)
        self.active = still
        self._admit()  # freed room is used at once
        return out

    def close(self) -> None:
        for job, run, _ in self.active:
            self.backend.abandon(run)
            self.backend.destroy(run)
        self.active = []
        for runs in self.idle.values():
            for run in runs:
                self.backend.destroy(run)
        self.idle.clear()
        self.sizes.clear()
        self.used = 0
        self.backend.close()
