"""The library in a fresh process without PyTorch, bound to the HIP runtime it was built with.

PyTorch ships its own HIP runtime (same soname); a process that imports torch
first makes the library bind to that one, whose version differs from the
headers the library was compiled with.  By default (LAGMEAN_HIP_RUNTIME=own) the
binding does not import torch and the library binds its own runtime; every GPU
test, the smoke test and the benchmarks run so.  These tests start such a
process afresh: it must bind ROCm's runtime of the library's own version, give
the oracle's results at 1e-12 in a single and a batched run, and serve a mix
with 512^2 and 1024^2 members exactly as each request alone.
"""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

from gpu_util import OUTPUT_KEYS, compare_value, oracle_run, say

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, ROOT)
import paper_2208_02682_amd as L
from synth import workload
assert "torch" not in sys.modules
w = workload("sw64_fp64")
u, v, h = w.initial_state()
cfg = L.make_config(w.N, precision="fp64", dt=w.dt, nu8=w.nu8)
single = L.Run(cfg)
single.set_state(u, v, h)
single.begin_interval()
single.step(40)
single.end_interval()
a = single.outputs()
batched = L.Run(cfg)
batched.set_state(u, v, h)
batched.begin_interval()
with L.Batch() as b:
    b.add(batched, 40)
    while b.step(16):
        pass
    b.remove(batched)
batched.end_interval()
c = batched.outputs()
np.savez(OUT, **{"single_" + k.replace(":", "_"): x for k, x in a.items()},
         **{"batched_" + k.replace(":", "_"): x for k, x in c.items()})
print(json.dumps({"hip": L.hip_runtime(), "torch_loaded": "torch" in sys.modules}))
"""


def test_library_alone_binds_its_own_runtime_and_matches_the_oracle(tmp_path):
    out = tmp_path / "own.npz"
    env = dict(os.environ, LAGMEAN_HIP_RUNTIME="own")
    code = f"ROOT = {ROOT!r}\nOUT = {str(out)!r}\n" + CHILD
    say("child process without torch (LAGMEAN_HIP_RUNTIME=own)")
    p = subprocess.run([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=240)
    say(p.stdout[-2000:])
    assert p.returncode == 0, p.stdout[-4000:]
    info = json.loads(p.stdout.strip().splitlines()[-1])
    assert info["torch_loaded"] is False
    assert info["hip"]["same"], info["hip"]        # built and bound HIP minor versions agree
    assert not any("torch" in f for f in info["hip"]["runtime_files"]), info["hip"]
    from synth import workload
    w = workload("sw64_fp64")
    _, ref = oracle_run(w, steps_per_interval=40, n_intervals=1)
    g = np.load(out)
    for key in OUTPUT_KEYS:
        name = key.replace(":", "_")
        assert np.array_equal(g[f"single_{name}"], g[f"batched_{name}"]), key
        e = compare_value(key, g[f"single_{name}"], ref[0][key])
        assert e < 1e-12, (key, e)


SERVE_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, ROOT)
import paper_2208_02682_amd as L
from paper_2208_02682_amd.serve import Job, Server
from synth.workloads import scaled_run
assert "torch" not in sys.modules
spec = [(1024, "fp32", 12), (512, "fp32", 20), (128, "fp32", 30), (1024, "fp32", 7), (256, "fp32", 16),
        (512, "fp64", 9), (128, "fp32", 11)]
reqs = [(scaled_run(N, Ro=0.05 + 0.01 * i, ratio=1.0, periods=1.0, seeds=(700 + 2 * i, 701 + 2 * i),
                    precision=p), n) for i, (N, p, n) in enumerate(spec)]
cfg = lambda w: L.make_config(w.N, precision=w.precision, dt=w.dt, nu8=w.nu8)
alone = []
for w, n in reqs:
    with L.Run(cfg(w)) as run:
        run.set_state(*w.initial_state())
        run.begin_interval()
        run.step(n)
        run.end_interval()
        alone.append(run.outputs())
# room for two 1024^2 runs and a little more: requests queue and runs are reused
budget = 2 * L.footprint(cfg(reqs[0][0])) + 3 * L.footprint(cfg(reqs[1][0]))
server = Server(budget, tick_steps=5)
done = []
for i, (w, n) in enumerate(reqs):
    server.submit(Job(i, cfg(w), w.initial_state(), n, arrival=server.clock()))
    if i % 2 == 1:
        done += server.tick()
while server.busy():
    done += server.tick()
server.close()
bad = [(j.id, k) for j in done for k in j.outputs if not np.array_equal(j.outputs[k], alone[j.id][k])]
print(json.dumps({"done": sorted(j.id for j in done), "errors": [j.error for j in done if j.error],
                  "mismatch": bad, "created": server.created}))
"""


def test_served_mix_with_512_and_1024_members_is_the_same_alone():
    """The serving loop on the library's own runtime (as the serving benchmark
    runs it) with 512^2 and 1024^2 members joining and leaving the batch: every
    request's outputs equal those of the same request run alone, bit for bit."""
    env = dict(os.environ, LAGMEAN_HIP_RUNTIME="own")
    code = f"ROOT = {ROOT!r}\n" + SERVE_CHILD
    say("served mix with 512^2 and 1024^2 members, child process without torch")
    p = subprocess.run([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=280)
    say(p.stdout[-2000:])
    assert p.returncode == 0, p.stdout[-4000:]
    res = json.loads(p.stdout.strip().splitlines()[-1])
    assert res["done"] == list(range(7)) and not res["errors"] and not res["mismatch"], res
