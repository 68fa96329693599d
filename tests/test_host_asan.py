"""Host-only sanitizer runs of the C ABI (no GPU).

The library's host code is built with AddressSanitizer and
UndefinedBehaviorSanitizer and linked to a stand-in HIP runtime
(tests/host_asan/hipstub.cpp) that keeps "device" memory in host memory and
defers every asynchronous copy, fill and kernel until its stream is waited for.
Scripts of C ABI calls are replayed through it (tests/host_asan/replay.cpp):

* a batch of runs of several sizes, precisions and options, as the batched
  tests drive it;
* the call sequence of the serving loop (paper_2208_02682_amd/serve.py, the
  real Server driving a recording backend) over a Poisson stream of averaging
  requests of N in {128, 256, 512, 1024}, with admission, pooling, eviction and
  a batch whose membership changes at every tick;
* the error paths (calls out of order, refused configurations).

Every run must finish with no sanitizer report.  A planted late copy into a
dead stack frame (tests/host_asan/late_copy.cpp) shows the harness detects the
class of mistake it is there for.
"""

import os
import subprocess

import pytest

from host_asan import harness

pytestmark = pytest.mark.skipif(not harness.available(), reason="hipcc / clang++ not installed")


@pytest.fixture(scope="module")
def exe():
    return harness.build()


def _clean(exe, script, name):
    rc, out = harness.replay(exe, script, name)
    assert rc == 0 and "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_batch_of_mixed_runs_is_clean(exe):
    lines = ["create 1 256 1 0.0025 0 0 0", "create 2 192 1 0.0033 1 0 0", "create 3 128 0 0.005 0 0 0",
             "create 4 128 1 0.005 0 40 0", "create 5 256 1 0.0025 0 7 0", "create 6 64 0 0.01 0 3 1"]
    for i in range(1, 7):
        lines += ([f"set {i}"] if i != 6 else []) + [f"begin {i}"]
    lines += ["batch"] + [f"add {i} {s}" for i, s in zip(range(1, 7), (40, 33, 27, 35, 21, 9))]
    lines += ["bstep 16"] * 3 + [f"remove {i}" for i in range(1, 7)] + ["bdestroy"]
    lines += [f"end {i}" for i in range(1, 7)] + ["remap 3", "state 1", "peek 2", "state 6"]
    # checkpoints: mid-interval and of a kinematic run, restored into fresh runs
    lines += ["begin 1", "step 1 3", "save 1", "create 7 256 1 0.0025 0 0 0", "restore 7 1", "step 7 2", "end 7",
              "save 6", "create 8 64 0 0.01 0 3 1", "restore 8 6", "expect -1", "restore 8 1"]
    out = _clean(exe, "\n".join(lines) + "\n", "batch")
    assert "operations ok" in out


class _Recorder:
    """A serve.Server backend that writes the C ABI calls it stands for."""

    def __init__(self):
        from paper_2208_02682_amd.lagmean import footprint
        self.footprint = footprint
        self.lines = ["batch"]
        self.ids = 0
        self.members = set()

    def create(self, cfg):
        self.ids += 1
        self.lines.append(f"create {self.ids} {cfg.n} {cfg.precision} {cfg.dt!r} {cfg.interp} {cfg.avg_fields} "
                          f"{cfg.mode}")
        return self.ids

    def start(self, run, job):
        self.lines += [f"set {run}", f"begin {run}", f"add {run} {job.steps}"]
        self.members.add(run)

    def step(self, n):
        self.lines.append(f"bstep {n}")

    def finish(self, run, keep):
        self.lines += [f"remove {run}", f"end {run}"]
        self.members.discard(run)
        return 0.0, None

    def abandon(self, run):
        if run in self.members:
            self.lines.append(f"remove {run}")
            self.members.discard(run)

    def destroy(self, run):
        self.lines.append(f"destroy {run}")

    def close(self):
        self.lines.append("bdestroy")


def serve_script(rate=20.0, window=30.0, budget_gib=4.0, tick=32, max_points=8 * 1024 * 1024):
    """The serving loop's calls for a Poisson stream of requests, with a simulated
    clock (a tick of n steps takes n * resident points / 2e9 seconds)."""
    from paper_2208_02682_amd.lagmean import make_config
    from paper_2208_02682_amd.serve import Job, Server
    from synth.workloads import serving_requests
    reqs = serving_requests(rate=rate, duration=window, seed=7)
    clock = [0.0]
    rec = _Recorder()
    server = Server(int(budget_gib * 2**30), max_resident_points=max_points, tick_steps=tick, backend=rec,
                    clock=lambda: clock[0], keep_outputs=False)
    i = done = 0
    while done < len(reqs):
        while i < len(reqs) and reqs[i].arrival <= clock[0]:
            w = reqs[i].run
            server.submit(Job(i, make_config(w.N, precision="fp32", dt=w.dt, nu8=w.nu8), (None,),
                              w.steps_per_interval, arrival=reqs[i].arrival))
            i += 1
        if not server.busy():
            clock[0] = reqs[i].arrival
            continue
        pts = server.resident_points
        n_before = len(rec.lines)
        fin = server.tick()
        steps = sum(int(line.split()[1]) for line in rec.lines[n_before:] if line.startswith("bstep"))
        clock[0] += max(steps * (pts or server.resident_points) / 2e9, 1e-4)
        done += len(fin)
        assert not any(j.error for j in fin), [j.error for j in fin if j.error]
    server.close()
    return len(reqs), "\n".join(rec.lines) + "\n"


def test_serving_loop_call_sequence_is_clean(exe):
    n, script = serve_script()
    assert n > 500 and script.count("bstep") > 100 and script.count("destroy") > 0
    out = _clean(exe, script, "serve")
    assert "operations ok" in out


def test_error_paths_are_clean(exe):
    script = """
create 1 64 0 0.01 0 0 0
expect -2
begin 1
expect -2
end 1
set 1
expect -2
end 1
begin 1
expect -2
end 1
step 1 3
end 1
begin 1
batch
add 1 5
expect -2
destroy 1
expect -2
step 1 1
expect -2
add 1 5
bstep 2
remove 1
expect -1
remove 1
bdestroy
expect -6
create 2 100 0 0.01 0 0 0
expect -6
create 3 64 0 0.01 0 11 0
create 4 64 0 0.01 0 3 1
expect -2
set 4
destroy 1
destroy 4
"""
    out = _clean(exe, script, "errors")
    assert "operations ok" in out


def test_the_harness_detects_a_late_copy_into_a_dead_frame():
    harness.build()
    exe = os.path.join(harness.OUT, "late_copy")
    subprocess.run([harness.CLANG, "-O1", "-g", "-std=c++17", *harness.SAN_LINK, "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", os.path.join(harness.HERE, "late_copy.cpp"), "-L" + harness.OUT,
                    "-lhipstub", "-Wl,-rpath," + harness.OUT, "-o", exe], check=True)
    env = dict(os.environ)
    env.update(harness.ENV)
    p = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=60)
    assert p.returncode != 0 and "stack-use-after-return" in p.stdout, p.stdout[-2000:]
