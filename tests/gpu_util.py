"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same inputs."""

from __future__ import annotations

import sys

import numpy as np

from oracle.lagmean import Params, Run as OracleRun, relative_l2

OUTPUT_KEYS = ["S2_mean:h", "S2_mean:zeta", "S2_xi_x", "S2_xi_y", "S1_mean:h", "S1_mean:zeta",
               "S1_eta_x", "S1_eta_y", "E_mean:h", "E_mean:zeta"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_value(key: str, a: np.ndarray, b: np.ndarray, H: float = 1.0) -> float:
    """Relative L2 with heights compared as h - H."""
    if key.endswith(":h") or key == "h":
        return relative_l2(a - H, b - H)
    return relative_l2(a, b)


def oracle_run(w, steps_per_interval=None, n_intervals=None, u=None, v=None, h=None, interp="bilinear"):
    if u is None:
        u, v, h = w.initial_state()
    p = Params(N=w.N, dt=w.dt, f=w.f, g=w.g, H=w.H, nu8=w.nu8, interp=interp)
    r = OracleRun(p, u, v, h)
    spi = steps_per_interval or w.steps_per_interval
    ni = n_intervals or w.n_intervals
    return r, r.run_intervals(spi, ni)


def gpu_run(w, steps_per_interval=None, n_intervals=None, u=None, v=None, h=None, chunk=None, interp="bilinear"):
    from paper_2208_02682_amd import Run, make_config
    if u is None:
        u, v, h = w.initial_state()
    cfg = make_config(w.N, precision=w.precision, f=w.f, g=w.g, H=w.H, dt=w.dt, nu8=w.nu8, interp=interp)
    run = Run(cfg)
    run.set_state(u, v, h)
    spi = steps_per_interval or w.steps_per_interval
    ni = n_intervals or w.n_intervals
    results = []
    for _ in range(ni):
        run.begin_interval()
        left = spi
        while left > 0:
            k = min(left, chunk or left)
            run.step(k)
            left -= k
        run.end_interval()
        results.append(run.outputs())
    return run, results
