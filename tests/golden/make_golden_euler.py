"""Write stored expected values for the two-dimensional incompressible test
(section 4.1): runs ONLY the CPU float64 oracle (oracle/euler2d.py) on the
two-vortex initial vorticity (eq. (4.3)) over the whole interval (128^2,
dt = 0.005, T = 25), for bilinear and cubic semi-Lagrangian gathers, and stores
every output on a regular sub-grid (every stride-th point from offset (2, 1))
plus the full-grid L2 norms.

    python tests/golden/make_golden_euler.py

The output is tests/golden/euler2d_two_vortex_128.npz.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.euler2d import Euler2D  # noqa: E402
from synth.euler import EULER_TWO_VORTEX as W  # noqa: E402

OFFSET = (2, 1)
STRIDE = 2


def main():
    store = {"stride": STRIDE, "offset": np.array(OFFSET), "N": W.N, "steps": W.steps, "dt": W.dt}
    t0 = time.time()
    for interp in ("bilinear", "cubic"):
        e = Euler2D(W.N, W.dt, W.initial_vorticity(), interp=interp)
        e.begin_interval()
        for k in range(0, W.steps, 250):
            e.step(min(250, W.steps - k))
            print(f"{interp}: step {k + 250}/{W.steps} ({time.time() - t0:.0f} s)", flush=True)
        out = e.end_interval()
        for key, val in out.items():
            store[f"{interp}_{key}"] = val[OFFSET[0]::STRIDE, OFFSET[1]::STRIDE].copy()
            store[f"{interp}_{key}_norm"] = np.array(np.linalg.norm(val))
    path = os.path.join(HERE, f"{W.name}.npz")
    np.savez_compressed(path, **store)
    print(f"wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
