"""Served form on the GPU: requests that join and leave a running mix give
exactly what each gives alone; pooled runs are reused with fresh results."""

import numpy as np
import pytest

from gpu_util import OUTPUT_KEYS, say

pytestmark = pytest.mark.gpu


def _requests():
    from synth.workloads import scaled_run
    spec = [(64, "fp64", 19), (128, "fp32", 33), (64, "fp32", 8), (128, "fp32", 21), (192, "fp32", 12),
            (64, "fp64", 27), (128, "fp64", 9), (64, "fp32", 15)]
    out = []
    for i, (N, prec, steps) in enumerate(spec):
        w = scaled_run(N, Ro=0.04 + 0.01 * i, ratio=0.5 + 0.25 * i, periods=1.0,
                       seeds=(300 + 2 * i, 301 + 2 * i), precision=prec)
        out.append((w, steps))
    return out


def _cfg(lib, w):
    return lib.make_config(w.N, precision=w.precision, dt=w.dt, nu8=w.nu8)


def test_each_request_is_the_same_alone_and_served():
    import paper_2208_02682_amd as lib
    from paper_2208_02682_amd.serve import Job, Server
    reqs = _requests()
    alone = []
    for w, steps in reqs:
        with lib.Run(_cfg(lib, w)) as run:
            run.set_state(*w.initial_state())
            run.begin_interval()
            run.step(steps)
            run.end_interval()
            alone.append(run.outputs())
    # a budget that holds about three of the larger runs: requests queue, runs
    # are reused and released, the mix changes between ticks
    budget = 3 * lib.footprint(_cfg(lib, reqs[4][0]))
    server = Server(budget, tick_steps=6)
    done = []
    try:
        for i, (w, steps) in enumerate(reqs):
            server.submit(Job(i, _cfg(lib, w), w.initial_state(), steps, arrival=server.clock()))
            if i % 3 == 2:
                done += server.tick()
        while server.busy():
            done += server.tick()
        # the configuration released last is idle in the pool: the same request
        # again reuses that run (no creation) and gives the same bits
        last = max(done, key=lambda j: j.finished)
        created = server.created
        w, steps = reqs[last.id]
        server.submit(Job(100 + last.id, _cfg(lib, w), w.initial_state(), steps, arrival=server.clock()))
        again = []
        while server.busy():
            again += server.tick()
        assert server.created == created and len(again) == 1 and again[0].error is None
        for k in OUTPUT_KEYS:
            assert np.array_equal(again[0].outputs[k], alone[last.id][k]), ("reused", last.id, k)
    finally:
        server.close()
    assert sorted(j.id for j in done) == list(range(len(reqs)))
    for j in done:
        assert j.error is None, j.error
        w, steps = reqs[j.id]
        assert j.T == pytest.approx(steps * w.dt, rel=1e-14)
        for k in OUTPUT_KEYS:
            assert np.array_equal(j.outputs[k], alone[j.id][k]), (j.id, w.N, w.precision, k)
    say(f"{len(reqs)} requests identical alone and served; {server.created} runs created, "
        f"{server.evicted} released")
