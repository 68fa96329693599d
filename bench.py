#!/usr/bin/env python3
"""Throughput of the coupled shallow-water + Lagrangian-mean step on one MI355X.

A step is one classical RK4 step of the whole hot path: the rotating
shallow-water dynamics and, in the same stages, strategy 1 (g-tilde and P),
strategy 2 (xi and g-bar) and the Eulerian accumulators, on the 1024 x 1024
turbulence-plus-waves workload (float32 transforms, float64 xi/P state).
The metric is grid-point RK4 steps per second (N^2 * steps / time), inputs
resident in HBM when the timed region starts.

Prints one JSON line with the driver's keys plus
  roofline     : the dominant kernel's algorithmic bytes per launch / its average
                 duration (HIP events on the run's stream), against 8 TB/s;
  cpu_baseline : the float64 CPU oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sw1024_fp32_hbm_traffic.md")
KERNEL_SOURCES = ["fft_core.hpp", "layout.hpp", "step_kernels.hpp"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2208_02682_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary, or
    None when it was taken for other kernel sources or another workload."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        parts = line.strip().split()
        if len(parts) >= 2 and parts[0].endswith(":"):
            fields[parts[0][:-1]] = parts[1]
    if fields.get("source_sha256") != kernel_source_hash() or fields.get("workload") != workload:
        return None
    v = fields.get(f"traffic_bytes_{kernel}")
    return float(v) if v is not None else None


def algorithmic_bytes(N: int, fp32: bool):
    """Compulsory bytes per launch of the three hot kernels (each input element
    read once, each output element written once), averaged over the 4 stages."""
    K = (N - 1) // 3
    nkx, nky = K + 1, 2 * K + 1
    cT = 8 if fp32 else 16          # complex element of the working precision
    rT = 4 if fp32 else 8
    cD = 16
    rowfield = N * nkx * cT         # one column-pass / row-pass field
    phys4 = N * N * 4 * rT          # interleaved u, v, eta, zeta
    sp = nkx * nky
    state = sp * (9 * cT + 4 * cD)  # 13 prognostic fields (xi, P in float64)
    rows_dyn = 4 * rowfield + phys4 + 5 * rowfield
    rows_rhs = 16 * rowfield + phys4 + 8 * rowfield
    # columns: 13 row spectra in, 20 column-pass outputs out, state Y read,
    # accumulator read (stages 2-4) and written (stages 1-3), Y written (stage 4),
    # stage values of u, v, h read and written
    columns = 13 * rowfield + 20 * rowfield + (1.0 + 0.75 + 0.75 + 0.25) * state + 6 * sp * cT
    return {"rows_dyn": rows_dyn, "rows_rhs": rows_rhs, "columns": columns}


def cpu_baseline(w, seconds: float):
    """The float64 oracle stepping the same initial state until ~seconds elapse."""
    from oracle import lagmean as olm
    threads = min(16, os.cpu_count() or 1)
    olm.set_workers(threads)
    u, v, h = w.initial_state()
    r = olm.Run(olm.Params(N=w.N, dt=w.dt, f=w.f, g=w.g, H=w.H, nu8=w.nu8), u, v, h)
    r.begin_interval()
    r.step(1)  # warm-up
    t0 = time.perf_counter()
    n = 0
    while True:
        r.step(1)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": w.N * w.N * n / el, "unit": "grid-pt RK4 steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} RK4 steps of the {w.N}^2 workload in float64 from its initial state "
                      f"({el:.1f} s, scipy.fft with {threads} threads)"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="sw1024_fp32")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the event-timed replay (roofline fields become null)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (the method's runs are independent per GPU); "
              f"--gpus {a.gpus} is not supported", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    if a.copy_probe:
        n = a.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 4, "repeats": 5}), flush=True)
        return 0
    from paper_2208_02682_amd import Run, make_config
    from synth import workload

    w = workload(a.workload)
    fp32 = w.precision == "fp32"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    u, v, h = w.initial_state()
    fields = [torch.from_numpy(x).cuda() for x in (u, v, h)]
    run = Run(make_config(w.N, precision=w.precision, f=w.f, g=w.g, H=w.H, dt=w.dt, nu8=w.nu8),
              stream=stream.cuda_stream)

    def start():
        run.set_state(*fields)
        run.begin_interval()
        run.step(a.warmup)
        torch.cuda.synchronize()

    # timed region: K plain steps from a fixed state (inputs resident in HBM)
    start()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    run.step(a.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)

    # the same K steps replayed from the same state with HIP events around every
    # launch (the kernels' cost depends on the state: the gathers spread as the
    # displacements grow), giving each kernel's average duration
    start()
    kms = [0.0, 0.0, 0.0]
    done = a.steps if a.no_kernel_timing else 0
    while done < a.steps:
        n = min(500, a.steps - done)
        part = run.step_profiled(n)
        kms = [x + y * n for x, y in zip(kms, part)]
        done += n
    kms = [x / a.steps for x in kms]
    T = run.end_interval()
    if a.no_kernel_timing:
        kms = [float("nan")] * 3
    names = ["rows_dyn", "rows_rhs", "columns"]
    ab = algorithmic_bytes(w.N, fp32)
    kernels = {n: {"avg_ms": kms[i], "alg_bytes": ab[n], "GBps": ab[n] / (kms[i] * 1e-3) / 1e9}
               for i, n in enumerate(names)}
    dom = max(names, key=lambda n: kernels[n]["avg_ms"]) if not a.no_kernel_timing else "columns"
    achieved = kernels[dom]["GBps"] if not a.no_kernel_timing else None
    step_bytes = 4 * sum(ab.values())

    pts = w.N * w.N
    value = pts * a.steps / (ms * 1e-3)
    rec = {
        "metric": "grid-pt RK4 steps/s incl. mean PDEs @1024^2",
        "value": value,
        "unit": "grid-pt RK4 steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: rotating shallow water {w.N}x{w.N} with strategy-1, strategy-2 "
                               f"and Eulerian means of h and zeta in the same RK4 stages",
                   "N": w.N, "precision": "float32 transforms/products/gathers, float64 xi and P state"
                   if fp32 else "float64", "dt": w.dt, "nu8": w.nu8, "steps_per_interval": w.steps_per_interval,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic(dom, w.name),
                     "alg_bytes_per_launch": kernels[dom]["alg_bytes"], "avg_launch_ms": kernels[dom]["avg_ms"]},
        "kernels": kernels,
        "step_alg_bytes_per_point": step_bytes / pts,
        "step_hbm_frac": step_bytes * a.steps / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "interval_T_partial": T,
    }
    if not a.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    run.close()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
