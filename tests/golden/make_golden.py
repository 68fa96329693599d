"""Write stored expected values for the full-size parity tests.

Runs ONLY the CPU float64 oracle (oracle/) on the seeded synthetic inputs of a
workload over all of its averaging intervals and stores, for every interval
and every output, the values on a regular sub-grid (every ``stride``-th point
in x and y, starting at (1, 2) so that the x and y samples differ), plus the
full-grid L2 norm of each output (heights as h - H).

    python tests/golden/make_golden.py sw256_fp64 --stride 8
    python tests/golden/make_golden.py sw1024recipe_at256_fp32 --stride 8
    python tests/golden/make_golden.py sw1024_fp32 --stride 16 --threads 6

The output is tests/golden/<workload>.npz.
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import lagmean as olm  # noqa: E402
from synth import workload  # noqa: E402

OFFSET = (2, 1)  # (row, column) of the first sample


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--stride", type=int, default=8)
    ap.add_argument("--threads", type=int, default=8)
    a = ap.parse_args(argv)
    olm.set_workers(a.threads)
    w = workload(a.workload)
    u, v, h = w.initial_state()
    r = olm.Run(olm.Params(N=w.N, dt=w.dt, f=w.f, g=w.g, H=w.H, nu8=w.nu8), u, v, h)
    store = {"stride": a.stride, "offset": np.array(OFFSET), "N": w.N,
             "steps_per_interval": w.steps_per_interval, "n_intervals": w.n_intervals}
    t0 = time.time()
    for i in range(w.n_intervals):
        r.begin_interval()
        for k in range(w.steps_per_interval):
            r.step(1)
            if k % 200 == 0:
                print(f"interval {i} step {k}/{w.steps_per_interval} ({time.time() - t0:.0f} s)", flush=True)
        out = r.end_interval()
        for key, val in out.items():
            name = key.replace(":", "_")
            store[f"i{i}_{name}"] = val[OFFSET[0]::a.stride, OFFSET[1]::a.stride].copy()
            ref = val - w.H if key.endswith(":h") else val
            store[f"i{i}_{name}_norm"] = np.array(np.linalg.norm(ref))
    path = os.path.join(HERE, f"{w.name}.npz")
    np.savez_compressed(path, **store)
    print(f"wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
