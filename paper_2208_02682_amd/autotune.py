"""Autotuner driver: the launch schedule of every (N, precision) is chosen by
timing the candidates on the device (lm_autotune, through Run.autotune) and the
choices are kept in a JSON cache per device architecture.

A schedule is the column-tile width of the column pass and the block order
(XCD-aware or hardware); every schedule computes the same numbers, so a cache
changes speed only.  Single runs and batched launches have separate tables
(tune: single runs, one at a time; tune_batch: the batched launches, on a
batch of runs).  The cache shipped with the package, schedules_gfx950.json,
holds the choices measured on an MI355X; load_default() applies it.
"""

from __future__ import annotations

import json
import os
from typing import Callable, Iterable, List, Optional, Tuple

from .lagmean import Config, Run, load_schedules, save_schedules

HERE = os.path.dirname(os.path.abspath(__file__))


def cache_path(arch: str) -> str:
    return os.path.join(HERE, f"schedules_{arch}.json")


def device_arch() -> str:
    """Architecture name of the first GPU (e.g. gfx950), from the kernel driver's
    topology (host only: no HIP call); "unknown" when the topology is not
    readable (then no cache matches and the default schedules stay)."""
    import glob
    for props in sorted(glob.glob("/sys/class/kfd/kfd/topology/nodes/*/properties")):
        try:
            with open(props) as f:
                kv = dict(line.split()[:2] for line in f if len(line.split()) >= 2)
        except OSError:
            continue
        v = int(kv.get("gfx_target_version", "0"))
        if v > 0:  # major * 10000 + minor * 100 + stepping; CPU nodes report 0
            return f"gfx{v // 10000}{(v // 100) % 100:x}{v % 100:x}"
    return "unknown"


def load_default(arch: Optional[str] = None) -> int:
    """Apply the shipped cache of the device's architecture; returns the number of
    (N, precision) schedules applied (0 if there is no cache for it)."""
    arch = arch or device_arch()
    path = cache_path(arch)
    if not os.path.exists(path):
        return 0
    return load_schedules(path, arch)


def tune(specs: Iterable[Tuple[int, str]], config_for: Callable[[int, str], Config],
         state_for: Callable[[int], tuple], *, warm_steps: int = 20, steps: int = 64, reps: int = 5) -> List[dict]:
    """Autotune every (N, precision) of specs on a run made with config_for(N,
    precision) from the state state_for(N), after warm_steps steps of an open
    interval (so that the strategy-2 gathers reach as far as in a running
    interval).  Each choice is applied as it is made; returns Run.autotune's
    records."""
    out = []
    for N, prec in specs:
        with Run(config_for(N, prec)) as r:
            r.set_state(*state_for(N))
            r.begin_interval()
            r.step(warm_steps)
            out.append(r.autotune(steps, reps))
    return out


def tune_batch(runs: List[Run], *, warm_steps: int = 20, steps: int = 8, reps: int = 5) -> List[dict]:
    """Autotune the batched launches' schedules on runs (each with a state; an
    interval is opened here and warm_steps steps taken first): they join one
    batch, lm_batch_autotune tunes every (N, precision) among them, and the
    batch is released.  The runs keep their state, with the interval open."""
    from .lagmean import Batch
    for r in runs:
        r.begin_interval()
        r.step(warm_steps)
    with Batch() as b:
        for r in runs:
            b.add(r, 1)
        out = b.autotune(steps, reps)
        for r in runs:
            b.remove(r)
    return out


def merge_save(path: str, arch: str, tuned: List[dict]) -> None:
    """Write tuned records to path, keeping the entries of other (context, N,
    precision) already there for the same architecture."""
    def key(t):
        return (t.get("context", "single"), t["n"], t["precision"])
    keep = []
    if os.path.exists(path):
        with open(path) as f:
            doc = json.load(f)
        if doc.get("format") == 1 and doc.get("arch") == arch:
            new = {key(t) for t in tuned}
            for e in doc["entries"]:
                if key(e) not in new:
                    keep.append({"context": e.get("context", "single"), "n": e["n"], "precision": e["precision"],
                                 "best": (e["col_tile"], e["xcd_order"], e.get("streams", 1)),
                                 "ms": {tuple(int(x) for x in k.split(",")): v for k, v in e["ms_per_step"].items()}})
    recs = sorted(keep + list(tuned), key=key)
    save_schedules(path, arch, recs)
