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

Three more modes print one JSON line each:
  --mode batch : 64 independent runs of uneven N (128..512, float32 transforms)
                 advanced together by one lm_batch, against the same runs one
                 after another alone and as plain float64 runs;
  --mode serve : Poisson arrivals of averaging requests (N in 128..1024) served
                 with admission by HBM footprint and continuous batching: p50/p99
                 latency from arrival to means on the host, at the offered rate
                 and at a sustainable rate (offered load 0.7 of the measured capacity);
  --mode euler : the two-dimensional incompressible test (two vortices, 128^2,
                 T = 25) with strategy 1 pseudospectral and semi-Lagrangian, and
                 the semi-Lagrangian kernel at 1024^2 against HBM;
  --mode tune  : the autotuner over every grid size and precision, written to the
                 schedule cache (paper_2208_02682_amd/schedules_<arch>.json);
  --mode latency : p50/p99 solve latency of the serving mix's requests served one
                 at a time (state handed over -> all means on the host).
Every mode applies the shipped schedule cache first (--no-schedule-cache: the
default schedules); --autotune measures the mode's own sizes first.
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
KERNEL_SOURCES = ["fft_core.hpp", "col_tile.hpp", "layout.hpp", "step_kernels.hpp"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2208_02682_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str, schedule=None):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE summary, or
    None when it was taken for other kernel sources, another workload or another
    launch schedule."""
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
    if schedule is not None and fields.get("schedule") != f"{schedule[0]},{schedule[1]}":
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
    # stage values of u, v, h read and written; float32 state also reads and
    # writes its trailing words in stage 4 (compensated RK4 update)
    comp = compensation_bytes(N) if fp32 else 0.0
    columns = 13 * rowfield + 20 * rowfield + (1.0 + 0.75 + 0.75 + 0.25) * state + 6 * sp * cT + comp
    return {"rows_dyn": rows_dyn, "rows_rhs": rows_rhs, "columns": columns}


def compensation_bytes(N: int) -> float:
    """Bytes per column launch (averaged over the 4 stages) of the trailing words
    of the compensated float32 state: 9 fields, read and written in stage 4."""
    K = (N - 1) // 3
    sp = (K + 1) * (2 * K + 1)
    return (0.25 + 0.25) * 9 * sp * 8


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


def _initial_state(w):
    return w.initial_state()


def generate_states(workloads, workers: int = 16):
    """Initial states of the requests, made on the host before any clock starts
    (worker processes; the GPU is not touched)."""
    import concurrent.futures
    import multiprocessing
    n = max(1, min(workers, os.cpu_count() or 1))
    with concurrent.futures.ProcessPoolExecutor(n, mp_context=multiprocessing.get_context("spawn")) as ex:
        return list(ex.map(_initial_state, workloads, chunksize=4))


def _cfg(w, precision=None):
    from paper_2208_02682_amd import make_config
    return make_config(w.N, precision=precision or w.precision, f=w.f, g=w.g, H=w.H, dt=w.dt, nu8=w.nu8)


def apply_schedules(a, specs, config_for, state_for) -> str:
    """Launch schedules for this run: the shipped cache of the device's
    architecture (unless --no-schedule-cache), then, with --autotune, fresh
    measurements of specs ((N, precision) pairs), saved to --schedules-out if
    given.  Returns where the schedules came from."""
    from paper_2208_02682_amd import autotune as at
    arch = at.device_arch()
    source = "default"
    if not a.no_schedule_cache and at.load_default(arch):
        source = "cache"
    if a.autotune:
        tuned = at.tune(specs, config_for, state_for)
        source = "autotune"
        for t in tuned:
            print(f"autotune: N={t['n']} {t['precision']}: best {t['best']} "
                  + ", ".join(f"{k}: {v:.4f} ms" for k, v in t["ms"].items()), file=sys.stderr, flush=True)
        if a.schedules_out:
            at.merge_save(a.schedules_out, arch, tuned)
    return source


def tune_batched(a, ws, states):
    """With --autotune: the batched launches' schedules, measured on a batch of
    the given runs (lm_batch_autotune), saved to --schedules-out if given."""
    if not a.autotune:
        return
    from paper_2208_02682_amd import Run
    from paper_2208_02682_amd import autotune as at
    runs = [Run(_cfg(w)) for w in ws]
    try:
        for r, st in zip(runs, states):
            r.set_state(*st)
        tuned = at.tune_batch(runs)
    finally:
        for r in runs:
            r.close()
    for t in tuned:
        print(f"autotune (batched): N={t['n']} {t['precision']}: {t['best']}", file=sys.stderr, flush=True)
    if a.schedules_out:
        at.merge_save(a.schedules_out, at.device_arch(), tuned)


def bench_tune(a) -> dict:
    """The autotuner over every grid size and precision; writes the cache."""
    from paper_2208_02682_amd import autotune as at
    from synth.workloads import scaled_run
    sizes = (64, 128, 192, 256, 384, 512, 1024)
    ws = {N: scaled_run(N, Ro=0.1, ratio=1.0, periods=1.0, seeds=(5, 6)) for N in sizes}
    states = dict(zip(sizes, generate_states([ws[N] for N in sizes])))
    specs = [(N, p) for N in sizes for p in ("fp32", "fp64")]
    a.autotune, a.no_schedule_cache = True, True
    if not a.schedules_out:
        a.schedules_out = at.cache_path(at.device_arch())
    t0 = time.perf_counter()
    apply_schedules(a, specs, lambda N, p: _cfg(ws[N], p), lambda N: states[N])
    # the batched launches: the 64 uneven runs of the batched workload
    from synth.workloads import batch_workloads
    bws = batch_workloads(a.batch_runs)
    tune_batched(a, bws, generate_states(bws))
    from paper_2208_02682_amd import get_schedule
    return {"mode": "tune", "arch": at.device_arch(), "seconds": time.perf_counter() - t0,
            "cache": os.path.relpath(a.schedules_out, ROOT),
            "schedules": {f"{N}:{p}": list(get_schedule(N, p)) for N, p in specs},
            "batched_schedules": {f"{N}:fp32": list(get_schedule(N, "fp32", batched=True))
                                  for N in sorted({w.N for w in bws})}}


def bench_batch(a) -> dict:
    """Config of 64 uneven runs: batched against alone, and against float64 alone."""
    import numpy as np
    from paper_2208_02682_amd import OUTPUTS, Batch, Run, device_synchronize
    from synth.workloads import batch_workloads

    ws = batch_workloads(a.batch_runs)
    states = generate_states(ws)
    pts = sum(w.N * w.N * w.steps_per_interval for w in ws)
    first = {}
    for w, st in zip(ws, states):
        first.setdefault(w.N, (w, st))
    sizes = sorted(first)
    source = apply_schedules(a, [(N, p) for N in sizes for p in ("fp32", "fp64")],
                             lambda N, p: _cfg(first[N][0], p), lambda N: first[N][1])
    tune_batched(a, ws, states)
    from paper_2208_02682_amd import get_schedule

    def start(run, st):
        run.set_state(*st)
        run.begin_interval()

    # warm-up of every distinct configuration (first launches, allocations)
    for prec in ("fp32", "fp64"):
        seen = set()
        for w, st in zip(ws, states):
            if w.N in seen:
                continue
            seen.add(w.N)
            with Run(_cfg(w, prec)) as r:
                start(r, st)
                r.step(2)
                r.end_interval()

    # batched: every run resident, one lm_batch until all budgets are spent,
    # then each interval closed (the division by T and the output transforms)
    runs = [Run(_cfg(w)) for w in ws]
    for r, st in zip(runs, states):
        start(r, st)
    device_synchronize()
    t0 = time.perf_counter()
    with Batch() as b:
        for r, w in zip(runs, ws):
            b.add(r, w.steps_per_interval)
        while b.step(a.tick_steps):
            pass
        for r in runs:
            b.remove(r)
    for r in runs:
        r.end_interval()
    t_batch = time.perf_counter() - t0
    batched = [r.outputs() for r in runs]
    for r in runs:
        r.close()

    def sequential(prec, compare):
        total = 0.0
        same = True
        for i, (w, st) in enumerate(zip(ws, states)):
            with Run(_cfg(w, prec)) as r:
                start(r, st)
                device_synchronize()
                t = time.perf_counter()
                r.step(w.steps_per_interval)
                r.end_interval()
                total += time.perf_counter() - t
                if compare:
                    o = r.outputs()
                    same = same and all(np.array_equal(o[k], batched[i][k]) for k in OUTPUTS)
        return total, same

    print(f"batch: {len(ws)} runs batched in {t_batch:.2f} s", file=sys.stderr, flush=True)
    t_alone, identical = sequential("fp32", True)
    print(f"batch: the same runs alone in {t_alone:.2f} s", file=sys.stderr, flush=True)
    t_fp64, _ = sequential("fp64", False)
    print(f"batch: float64 runs alone in {t_fp64:.2f} s", file=sys.stderr, flush=True)
    return {
        "metric": f"aggregate grid-pt RK4 steps/s, {len(ws)} uneven runs batched", "value": pts / t_batch,
        "unit": "grid-pt RK4 steps/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{len(ws)} independent runs, N in {sizes}, float32 transforms with float64 "
                               f"xi and P, Ro ~ U[0.02, 0.2], wave/vortex energy ratio log-U[0.25, 4], "
                               f"T ~ U[1, 8] wave periods, dt = 0.64/N",
                   "runs": len(ws), "total_steps": sum(w.steps_per_interval for w in ws),
                   "grid_point_steps": pts, "tick_steps": a.tick_steps,
                   "schedules": {f"{N}:{p}": list(get_schedule(N, p)) for N in sizes for p in ("fp32", "fp64")},
                   "batched_schedules": {f"{N}:fp32": list(get_schedule(N, "fp32", batched=True)) for N in sizes},
                   "schedule_source": source},
        "seconds": {"batched": t_batch, "alone_sequential": t_alone, "fp64_alone_sequential": t_fp64},
        "alone_sequential_value": pts / t_alone, "fp64_alone_sequential_value": pts / t_fp64,
        "speedup_vs_alone": t_alone / t_batch, "speedup_vs_fp64_alone": t_fp64 / t_batch,
        "batched_identical_to_alone": identical,
    }


def _serve_once(reqs, states, rate, window, a, t_limit):
    """Real-time serving of one arrival sequence; returns the per-request timings."""
    import numpy as np
    from paper_2208_02682_amd.serve import Job, Server

    server = Server(a.hbm_budget_gib * 2**30, max_resident_points=a.max_resident_points,
                    tick_steps=a.tick_steps)
    # resident state: one run of every configuration created and warmed up
    # before the clock starts (later requests reuse pooled runs)
    seen = {}
    for r, st in zip(reqs, states):
        seen.setdefault(r.run.N, (r.run, st))
    for i, (w, st) in enumerate(seen.values()):
        server.submit(Job(-1 - i, _cfg(w), st, 2, arrival=server.clock()))
    while server.busy():
        server.tick()
    done, lat = [], {}
    busy = 0.0
    t0 = time.perf_counter()
    i = 0
    while len(done) < len(reqs):
        now = time.perf_counter() - t0
        if now > t_limit:
            break
        while i < len(reqs) and reqs[i].arrival <= now:
            r = reqs[i]
            server.submit(Job(r.index, _cfg(r.run), states[i], r.run.steps_per_interval, arrival=t0 + r.arrival))
            states[i] = None
            i += 1
        if not server.busy():
            if i < len(reqs):
                time.sleep(max(0.0, min(reqs[i].arrival - (time.perf_counter() - t0), 0.05)))
            continue
        tb = time.perf_counter()
        for j in server.tick():
            if j.error is not None:
                raise RuntimeError(f"request {j.id}: {j.error}")
            j.outputs = None  # the means reached the host; the benchmark does not keep them
            done.append(j)
            lat[j.id] = j.latency
            if len(done) % 50 == 0:
                print(f"serve: {len(done)}/{len(reqs)} requests done at {time.perf_counter() - t0:.1f} s, "
                      f"{len(server.queue)} queued, {len(server.active)} resident", file=sys.stderr, flush=True)
        busy += time.perf_counter() - tb
    elapsed = time.perf_counter() - t0
    stats = {"created_runs": server.created, "released_runs": server.evicted}
    server.close()
    size = {r.index: r.run.N * r.run.N * r.run.steps_per_interval for r in reqs}
    served = sum(size[j.id] for j in done)
    offered = sum(size.values()) / window
    capacity = served / busy if busy > 0 else float("nan")
    all_lat = np.array([lat.get(r.index, np.inf) for r in reqs])
    got = np.array(sorted(lat.values()))

    def pct(x, q):
        v = float(np.percentile(x, q)) if len(x) else float("nan")
        return v if np.isfinite(v) else None
    in_window = sum(1 for j in done if j.finished - t0 <= window)
    return {"rate_per_s": rate, "window_s": window, "requests": len(reqs), "completed": len(done),
            "completed_fraction": len(done) / len(reqs), "completed_within_window_fraction": in_window / len(reqs),
            "p50_latency_s": pct(all_lat, 50), "p99_latency_s": pct(all_lat, 99),
            "p50_latency_completed_s": pct(got, 50), "p99_latency_completed_s": pct(got, 99),
            "mean_latency_completed_s": float(got.mean()) if len(got) else None,
            "elapsed_s": elapsed, "offered_pt_steps_per_s": offered, "served_pt_steps_per_s": served / elapsed,
            "capacity_pt_steps_per_s": capacity, "rho": offered / capacity, **stats}


def _fp64_sequential(reqs, a) -> dict:
    """The same requests served one after another as plain float64 single runs:
    the first --fp64-sample requests of every grid size are run and timed (state
    handed over -> all means on the host), which gives each size's float64
    service rate; the first-come-first-served latency of a sequential float64
    server over the whole arrival sequence then follows from those measured
    rates (each request's service time = its grid-point steps / its size's rate)."""
    import numpy as np
    from paper_2208_02682_amd import Run
    per_n = {}
    for r in reqs:
        per_n.setdefault(r.run.N, [])
        if len(per_n[r.run.N]) < a.fp64_sample:
            per_n[r.run.N].append(r)
    rate, measured = {}, 0
    for N, sample in sorted(per_n.items()):
        states = generate_states([r.run for r in sample])
        with Run(_cfg(sample[0].run, "fp64")) as run:
            run.set_state(*states[0])  # warm-up
            run.begin_interval()
            run.step(2)
            run.end_interval()
            work, t_all = 0, 0.0
            for r, st in zip(sample, states):
                t0 = time.perf_counter()
                run.set_state(*st)
                run.begin_interval()
                run.step(r.run.steps_per_interval)
                run.end_interval()
                out = run.outputs()
                t_all += time.perf_counter() - t0
                work += r.run.N * r.run.N * r.run.steps_per_interval
                assert all(np.isfinite(v).all() for v in out.values())
        rate[N] = work / t_all
        measured += len(sample)
        print(f"serve: float64 sequential, N={N}: {len(sample)} requests at {rate[N]:.3e} pt-steps/s",
              file=sys.stderr, flush=True)
    free, lat = 0.0, []
    for r in reqs:
        svc = r.run.N * r.run.N * r.run.steps_per_interval / rate[r.run.N]
        start = max(free, r.arrival)
        free = start + svc
        lat.append(free - r.arrival)
    lat = np.array(lat)
    total = sum(r.run.N * r.run.N * r.run.steps_per_interval for r in reqs)
    busy = sum(r.run.N * r.run.N * r.run.steps_per_interval / rate[r.run.N] for r in reqs)
    return {"measured_requests": measured, "sample_per_size": a.fp64_sample,
            "pt_steps_per_s_by_N": {str(N): v for N, v in sorted(rate.items())},
            "capacity_pt_steps_per_s": total / busy,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "note": "latencies of a first-come-first-served sequential float64 server over the same arrivals, "
                    "from the service rates measured on the sampled requests"}


def bench_serve(a) -> dict:
    import numpy as np
    from paper_2208_02682_amd import hip_runtime
    from synth.workloads import serving_requests

    reqs = serving_requests(rate=a.rate, duration=a.window, seed=7)
    sizes = sorted({r.run.N for r in reqs})
    states = generate_states([r.run for r in reqs])
    print(f"serve: {len(reqs)} request states generated", file=sys.stderr, flush=True)
    first = {}
    for r, st in zip(reqs, states):
        first.setdefault(r.run.N, (r.run, st))
    source = apply_schedules(a, [(N, "fp32") for N in sizes], lambda N, p: _cfg(first[N][0], p),
                             lambda N: first[N][1])
    mean_work = float(np.mean([r.run.N * r.run.N * r.run.steps_per_interval for r in reqs]))
    main = _serve_once(reqs, states, a.rate, a.window, a, a.window + a.drain_limit)
    rec = {"metric": "p50/p99 solve latency (arrival to means on the host), Poisson arrivals",
           "value": main["p99_latency_s"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": f"averaging requests, N in {sizes} with probabilities 0.4/0.3/0.2/0.1, the "
                                  f"64^2 recipe scaled to N, float32 transforms with float64 xi and P, "
                                  f"T ~ U[1, 8] wave periods, dt = 0.64/N, arrival seed 7",
                      "mean_grid_point_steps_per_request": mean_work, "hbm_budget_gib": a.hbm_budget_gib,
                      "max_resident_points": a.max_resident_points, "tick_steps": a.tick_steps,
                      "schedule_source": source},
           "hip": hip_runtime(),
           "offered": main}
    rec["fp64_sequential"] = _fp64_sequential(reqs, a)
    if a.sustainable_window > 0 and np.isfinite(main["capacity_pt_steps_per_s"]):
        rate = 0.7 * main["capacity_pt_steps_per_s"] / mean_work
        reqs2 = serving_requests(rate=rate, duration=a.sustainable_window, seed=7)
        states2 = generate_states([r.run for r in reqs2])
        rec["sustainable"] = _serve_once(reqs2, states2, rate, a.sustainable_window, a,
                                         a.sustainable_window + a.drain_limit)
    return rec


def bench_latency(a) -> dict:
    """Solve latency of averaging requests served one at a time (no batching,
    no queueing): for each request of the serving workload's mix, the time
    from handing over its initial state to having every mean on the host.
    Runs are pooled per configuration, as in serving; states are generated
    before any clock starts."""
    import numpy as np
    from paper_2208_02682_amd import Run
    from synth.workloads import serving_requests

    reqs = serving_requests(rate=20.0, duration=a.latency_window, seed=7)
    states = generate_states([r.run for r in reqs])
    sizes = sorted({r.run.N for r in reqs})
    first = {}
    for r, st in zip(reqs, states):
        first.setdefault(r.run.N, (r.run, st))
    source = apply_schedules(a, [(N, "fp32") for N in sizes], lambda N, p: _cfg(first[N][0], p),
                             lambda N: first[N][1])
    pool = {}
    for N in sizes:  # one run per grid size, created and warmed up before the clock starts
        w, st = first[N]
        run = Run(_cfg(w))
        run.set_state(*st)
        run.begin_interval()
        run.step(2)
        run.end_interval()
        pool[N] = run
    lat, work = [], 0
    t_all = time.perf_counter()
    for r, st in zip(reqs, states):
        run = pool[r.run.N]
        t0 = time.perf_counter()
        run.set_state(*st)
        run.begin_interval()
        run.step(r.run.steps_per_interval)
        run.end_interval()
        out = run.outputs()
        lat.append(time.perf_counter() - t0)
        work += r.run.N * r.run.N * r.run.steps_per_interval
        assert all(np.isfinite(v).all() for v in out.values())
    elapsed = time.perf_counter() - t_all
    for run in pool.values():
        run.close()
    lat = np.array(lat)
    by_n = {}
    for N in sizes:
        x = np.array([l for l, r in zip(lat, reqs) if r.run.N == N])
        by_n[str(N)] = {"requests": int(len(x)), "p50_s": float(np.percentile(x, 50)),
                        "p99_s": float(np.percentile(x, 99))}
    return {"metric": "p50/p99 solve latency, requests served one at a time", "value": float(np.percentile(lat, 99)),
            "unit": "s", "n_gpus": 1, "higher_is_better": False, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": f"averaging requests, N in {sizes} with probabilities 0.4/0.3/0.2/0.1, the "
                                   f"64^2 recipe scaled to N, float32 transforms with float64 xi and P, "
                                   f"T ~ U[1, 8] wave periods, dt = 0.64/N, seed 7, first {len(reqs)} requests",
                       "schedule_source": source},
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "requests": len(reqs), "by_N": by_n,
            "throughput_pt_steps_per_s": work / elapsed}


def bench_euler(a) -> dict:
    """The two-dimensional incompressible test of section 4.1 (128^2, dt 0.005,
    T = 25) with strategy 1 pseudospectral and semi-Lagrangian, plus the
    semi-Lagrangian kernel (FFT-free, gather-bound) at 1024^2 against HBM."""
    import numpy as np
    from paper_2208_02682_amd import Euler2D, device_synchronize
    from synth.euler import EULER_TWO_VORTEX as W, two_vortex_vorticity

    z0 = W.initial_vorticity()
    runs = {}
    for interp in ("bilinear", "cubic"):
        with Euler2D(W.N, W.dt, interp=interp) as e:
            e.set_vorticity(z0)
            e.begin_interval()
            e.step(10)                       # warm-up inside the interval
            e.set_vorticity(z0)
            e.begin_interval()
            device_synchronize()
            t0 = time.perf_counter()
            e.step(W.steps)
            e.end_interval()
            el = time.perf_counter() - t0
            out = e.outputs()
        rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))
        runs[interp] = {"seconds": el, "grid_point_steps_per_s": W.N * W.N * W.steps / el,
                        "material_conservation_rel_l2": {"pseudospectral": rel(out["PS_mean"], out["zeta"]),
                                                         "semi_lagrangian": rel(out["SL_mean"], out["zeta"])}}
        print(f"euler: {interp} interval in {el:.2f} s", file=sys.stderr, flush=True)
    # the semi-Lagrangian kernel at 1024^2: 3 inputs (u, v, zeta_{n+1}), 4 gathered
    # fields each read once, 4 outputs, float64
    N = 1024
    sl = {}
    for interp in ("bilinear", "cubic"):
        with Euler2D(N, 0.0025, interp=interp) as e:
            e.set_vorticity(two_vortex_vorticity(N))
            e.begin_interval()
            e.step(5)
            ms_step, ms_sl = e.step_profiled(100)
        ab = 11 * 8 * N * N
        sl[interp] = {"avg_ms": ms_sl, "alg_bytes": ab, "GBps": ab / (ms_sl * 1e-3) / 1e9,
                      "frac": ab / (ms_sl * 1e-3) / (HBM_PEAK_GBS * 1e9), "step_ms": ms_step}
    return {"metric": "grid-pt steps/s, 2-D incompressible flow with strategy 1 pseudospectral and semi-Lagrangian",
            "value": runs["cubic"]["grid_point_steps_per_s"], "unit": "grid-pt steps/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{W.name}: two Gaussian vortices (eq. (4.3)), N = {W.N}, dt = {W.dt}, "
                                   f"T = {W.T} ({W.steps} Heun steps), one interval; value = cubic gathers",
                       "N": W.N, "steps": W.steps},
            "runs": runs,
            "roofline": {"bound": "hbm", "kernel": "k_e2d_sl (1024^2, cubic)", "achieved": sl["cubic"]["GBps"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sl["cubic"]["frac"], "traffic": None},
            "sl_kernel_1024": sl}


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
    ap.add_argument("--mode", choices=("step", "batch", "serve", "euler", "tune", "latency"), default="step")
    ap.add_argument("--latency-window", type=float, default=3.0,
                    help="latency: requests of this many seconds of the 20 /s arrival sequence")
    ap.add_argument("--autotune", action="store_true",
                    help="measure the launch schedules of the mode's grid sizes first (lm_autotune)")
    ap.add_argument("--no-schedule-cache", action="store_true",
                    help="do not apply the shipped schedule cache (default schedules unless --autotune)")
    ap.add_argument("--schedules-out", default=None, metavar="PATH",
                    help="with --autotune (or --mode tune): write the choices to this JSON cache")
    ap.add_argument("--batch-runs", type=int, default=64)
    ap.add_argument("--tick-steps", type=int, default=32, help="batch/serve: steps per lm_batch_step call")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: arrivals per second")
    ap.add_argument("--window", type=float, default=30.0, help="serve: seconds of arrivals")
    ap.add_argument("--sustainable-window", type=float, default=60.0,
                    help="serve: seconds of arrivals at 0.7 of the measured capacity (0 = skip)")
    ap.add_argument("--drain-limit", type=float, default=300.0,
                    help="serve: seconds after the last arrival before unfinished requests are counted as such")
    ap.add_argument("--hbm-budget-gib", type=float, default=64.0)
    ap.add_argument("--fp64-sample", type=int, default=6,
                    help="serve: requests per grid size timed as plain float64 single runs")
    ap.add_argument("--max-resident-points", type=int, default=8 * 1024 * 1024)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (the method's runs are independent per GPU); "
              f"--gpus {a.gpus} is not supported", file=sys.stderr)
        return 2

    if a.mode == "serve":
        import faulthandler
        faulthandler.enable()
    if a.mode in ("batch", "serve", "euler", "tune", "latency"):
        rec = {"batch": bench_batch, "serve": bench_serve, "euler": bench_euler, "tune": bench_tune,
               "latency": bench_latency}[a.mode](a)
        print(json.dumps(rec), flush=True)
        return 0
    from paper_2208_02682_amd import DeviceArray, Run, copy_bandwidth, device_synchronize, hip_runtime, make_config
    if a.copy_probe:
        # a plain device copy of MIB MiB, five times (calibrates the counters)
        gbps = copy_bandwidth(a.copy_probe * (1 << 20), 5)
        print(json.dumps({"copy_probe_bytes_each_way": a.copy_probe * (1 << 20), "repeats": 5, "GBps": gbps}),
              flush=True)
        return 0
    from synth import workload

    w = workload(a.workload)
    fp32 = w.precision == "fp32"
    u, v, h = w.initial_state()
    fields = [DeviceArray.from_host(x) for x in (u, v, h)]
    source = apply_schedules(a, [(w.N, w.precision)], lambda N, p: _cfg(w, p), lambda N: (u, v, h))
    from paper_2208_02682_amd import get_schedule
    sched = get_schedule(w.N, w.precision)
    run = Run(make_config(w.N, precision=w.precision, f=w.f, g=w.g, H=w.H, dt=w.dt, nu8=w.nu8))

    def start():
        run.set_state(*fields)
        run.begin_interval()
        run.step(a.warmup)
        device_synchronize()

    # timed region: K plain steps from a fixed state (inputs resident in HBM),
    # between HIP events on the run's stream, the device idle before
    start()
    ms = run.step_timed(a.steps)

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
    # strategy 1 at mean positions (eq. (3.8)) for the interval just closed:
    # once per interval, not part of a step
    t0 = time.perf_counter()
    remap_res = run.remap_s1()
    remap_ms = (time.perf_counter() - t0) * 1e3
    if a.no_kernel_timing:
        kms = [float("nan")] * 3
    # measured bandwidth of a plain device copy (1 GiB read + 1 GiB written, five
    # times, HIP events), reported beside the published 8 TB/s
    copy_gbps = copy_bandwidth(1 << 30, 5)
    for f in fields:
        f.close()
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
        "metric": f"grid-pt RK4 steps/s incl. mean PDEs @{w.N}^2",
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
                   "parallelism": "single GPU",
                   "schedule": {"col_tile": sched[0], "xcd_order": sched[1], "streams": sched[2],
                                "source": source}},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic(dom, w.name, sched),
                     "alg_bytes_per_launch": kernels[dom]["alg_bytes"], "avg_launch_ms": kernels[dom]["avg_ms"],
                     "copy_probe_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps if achieved else None},
        "kernels": kernels,
        "hip": hip_runtime(),
        "step_alg_bytes_per_point": step_bytes / pts,
        "step_hbm_frac": step_bytes * a.steps / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
        "interval_T_partial": T,
        "remap_s1": {"ms": remap_ms, "residual_cells": remap_res,
                     "note": "lm_remap_s1 on the interval closed after the profiled pass (host wall clock, "
                             "synchronous call); once per interval, not in the step"},
    }
    if fp32:
        # the compensated float32 state: its trailing words are read and written
        # in stage 4 of the column pass (algorithmic bytes, per launch averaged
        # over the 4 stages, and per step)
        comp = compensation_bytes(w.N)
        rec["compensation"] = {"bytes_per_column_launch": comp, "bytes_per_step": 4 * comp,
                               "share_of_step_bytes": 4 * comp / step_bytes,
                               "ms_per_step_at_hbm_rate": 4 * comp / (step_bytes * a.steps / (ms * 1e-3)) * 1e3}
    if not a.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    run.close()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
