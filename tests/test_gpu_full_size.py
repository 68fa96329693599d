"""Full-size parity: whole multi-interval runs on the GPU against stored oracle values.

The stored values (tests/golden/<workload>.npz) were written by
tests/golden/make_golden.py, which runs only the CPU float64 oracle: every
output of every averaging interval on a regular sub-grid (every stride-th
point from the stored offset) and the full-grid L2 norm of each output.  The
GPU path runs the same workload through the C ABI, in the same launch
configuration bench.py uses, and is compared on the sampled points (relative
L2 over the samples, heights as h - H, positions as displacements).
"""

import os

import numpy as np
import pytest

from gpu_util import OUTPUT_KEYS, gpu_run, say

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _compare(name, tol):
    from synth import workload
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    g = np.load(path)
    w = workload(name)
    stride, off = int(g["stride"]), tuple(int(x) for x in g["offset"])
    assert int(g["steps_per_interval"]) == w.steps_per_interval and int(g["n_intervals"]) == w.n_intervals
    say(f"{name}: {w.n_intervals} x {w.steps_per_interval} steps on the GPU")
    run, got = gpu_run(w, chunk=512)
    worst = {}
    for i in range(w.n_intervals):
        for key in OUTPUT_KEYS:
            ref = g[f"i{i}_{key.replace(':', '_')}"]
            val = got[i][key][off[0]::stride, off[1]::stride]
            if key.endswith(":h"):
                ref, val = ref - w.H, val - w.H
            nb = np.linalg.norm(ref)
            err = np.linalg.norm(val - ref) / nb if nb > 1e-14 else np.max(np.abs(val - ref))
            worst[key] = max(worst.get(key, 0.0), err)
            say(f"  interval {i} {key}: rel {err:.3e}")
    run.close()
    return worst


def test_sw256_fp64_four_intervals():
    worst = _compare("sw256_fp64", 1e-12)
    for k, e in worst.items():
        assert e < 1e-12, (k, e)


def test_1024_recipe_at_256_mixed_two_intervals():
    """The mixed-precision path over a whole 2-interval run against float64."""
    worst = _compare("sw1024recipe_at256_fp32", 1e-5)
    for k, e in worst.items():
        assert e < 1e-5, (k, e)
