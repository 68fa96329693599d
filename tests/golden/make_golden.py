"""Write stored expected values for the full-size parity tests.

Runs ONLY the CPU float64 oracle (oracle/) on the seeded synthetic inputs of a
workload over all of its averaging intervals and stores, for every interval
and every output, the values on a regular sub-grid (every ``stride``-th point
in x and y, starting at (1, 2) so that the x and y samples differ), plus the
full-grid L2 norm of each output (heights as h - H).

    python tests/golden/make_golden.py sw256_fp64 --stride 8
    python tests/golden/make_golden.py sw1024recipe_at256_fp32 --stride 8
    python tests/golden/make_golden.py sw1024_fp32 --stride 4 --threads 6 --checkpoint /tmp/g1024.npz

The output is tests/golden/<workload>.npz.  With --checkpoint, the oracle's
state is saved every --checkpoint-every steps and a rerun resumes from it.
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


def save_checkpoint(path, r, i, k, store):
    """Oracle state (spectral fields and step counters), position and the values
    stored so far; written to a temporary file first, then renamed."""
    arrays = {"pos": np.array([i, k, r.n, r.n_tau], dtype=np.int64)}
    arrays.update({"Y__" + key.replace(":", "__c__"): val for key, val in r.Y.items()})
    arrays.update({"S__" + key: np.asarray(val) for key, val in store.items()})
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def load_checkpoint(path, r, store):
    with np.load(path) as z:
        i, k, n, n_tau = (int(x) for x in z["pos"])
        for name in z.files:
            if name.startswith("Y__"):
                r.Y[name[3:].replace("__c__", ":")] = z[name].copy()
            elif name.startswith("S__"):
                store[name[3:]] = z[name].copy()
    r.n, r.n_tau = n, n_tau
    return i, k


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--stride", type=int, default=8)
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--checkpoint-every", type=int, default=250)
    ap.add_argument("--intervals", type=int, default=0, help="store only the first K intervals (0 = all)")
    a = ap.parse_args(argv)
    olm.set_workers(a.threads)
    w = workload(a.workload)
    u, v, h = w.initial_state()
    r = olm.Run(olm.Params(N=w.N, dt=w.dt, f=w.f, g=w.g, H=w.H, nu8=w.nu8), u, v, h)
    n_int = min(a.intervals, w.n_intervals) if a.intervals > 0 else w.n_intervals
    store = {"stride": a.stride, "offset": np.array(OFFSET), "N": w.N,
             "steps_per_interval": w.steps_per_interval, "n_intervals": n_int}
    i0 = k0 = 0
    if a.checkpoint and os.path.exists(a.checkpoint):
        i0, k0 = load_checkpoint(a.checkpoint, r, store)
        store["n_intervals"] = n_int  # this invocation's count, whatever the checkpoint's was
        print(f"resumed at interval {i0} step {k0}", flush=True)
    t0 = time.time()
    for i in range(i0, n_int):
        if not (i == i0 and k0 > 0):
            r.begin_interval()
        for k in range(k0 if i == i0 else 0, w.steps_per_interval):
            r.step(1)
            if k % 200 == 0:
                print(f"interval {i} step {k}/{w.steps_per_interval} ({time.time() - t0:.0f} s)", flush=True)
            if a.checkpoint and (k + 1) % a.checkpoint_every == 0 and k + 1 < w.steps_per_interval:
                save_checkpoint(a.checkpoint, r, i, k + 1, store)
        out = r.end_interval()
        for key, val in out.items():
            name = key.replace(":", "_")
            store[f"i{i}_{name}"] = val[OFFSET[0]::a.stride, OFFSET[1]::a.stride].copy()
            ref = val - w.H if key.endswith(":h") else val
            store[f"i{i}_{name}_norm"] = np.array(np.linalg.norm(ref))
        if a.checkpoint:
            save_checkpoint(a.checkpoint, r, i + 1, 0, store)
    path = os.path.join(HERE, f"{w.name}.npz")
    np.savez_compressed(path, **store)
    print(f"wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
