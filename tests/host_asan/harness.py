"""Host-only sanitizer build of the C ABI against the stand-in HIP runtime.

Test infrastructure: compiles the library's host code (hipcc --cuda-host-only,
no device code) with AddressSanitizer and UndefinedBehaviorSanitizer, links it
to hipstub.cpp instead of the HIP runtime, and runs replay.cpp on scripts of
C ABI calls.  Everything runs on the CPU; nothing here is loaded by the GPU
path.  Objects go to _build/host_asan/ and are rebuilt when a source changes.
"""

from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2208_02682_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(ROOT, "_build", "host_asan")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
# sanitizers apply to host code only (-Xarch_host before each -fsanitize=)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
SAN_LINK = ["-fsanitize=address", "-fsanitize=undefined"]
ENV = {"ASAN_OPTIONS": "detect_stack_use_after_return=1:detect_leaks=0:abort_on_error=0:halt_on_error=1",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def available() -> bool:
    return os.path.exists(HIPCC) and os.path.exists(CLANG)


def _digest(paths) -> str:
    h = hashlib.sha256()
    for p in sorted(paths):
        with open(p, "rb") as f:
            h.update(p.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd[:3])} ... failed:\n{p.stdout[-4000:]}")


def build(jobs: int = 4) -> str:
    """Build (if needed) and return the path of the replay executable."""
    os.makedirs(OUT, exist_ok=True)
    hips = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    own = [os.path.join(HERE, f) for f in ("hipstub.cpp", "replay.cpp", "harness.py")]
    tag = _digest(hips + hdrs + own + [os.path.join(INCLUDE, "lagmean.h")])
    exe = os.path.join(OUT, f"replay_{tag}")
    if os.path.exists(exe):
        return exe
    stub = os.path.join(OUT, "libhipstub.so")
    _run([CLANG, "-shared", "-fPIC", "-O1", "-g", "-std=c++17", *SAN_LINK, "-D__HIP_PLATFORM_AMD__",
          "-I/opt/rocm/include", os.path.join(HERE, "hipstub.cpp"), "-o", stub])

    def obj(src):
        o = os.path.join(OUT, os.path.basename(src)[:-4] + ".o")
        _run([HIPCC, "--offload-arch=gfx950", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC", *SAN,
              "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", o])
        return o

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(obj, hips))
    # a host-only object refers to its translation unit's device image
    # (__hip_fatbin_<hash>), which only a device compile makes: stand-ins here
    fat = set()
    for o in objs:
        p = subprocess.run(["nm", "-u", o], stdout=subprocess.PIPE, text=True, check=True)
        fat.update(line.split()[-1] for line in p.stdout.splitlines() if "__hip_fatbin" in line)
    fat_src = os.path.join(OUT, "fatbins.c")
    with open(fat_src, "w") as f:
        f.write("".join(f"char {name}[16];\n" for name in sorted(fat)))
    fat_obj = os.path.join(OUT, "fatbins.o")
    _run([CLANG, "-x", "c", "-c", "-fPIC", fat_src, "-o", fat_obj])
    lib = os.path.join(OUT, "liblagmean_asan.so")
    _run([CLANG, "-shared", "-fPIC", *SAN_LINK, *objs, fat_obj, "-L" + OUT, "-lhipstub", "-Wl,-rpath," + OUT,
          "-o", lib])
    _run([CLANG, "-O1", "-g", "-std=c++17", *SAN_LINK, "-I", INCLUDE, os.path.join(HERE, "replay.cpp"), lib,
          "-Wl,-rpath," + OUT, "-o", exe])
    return exe


def replay(exe: str, script: str, name: str = "script"):
    """Run a script; returns (returncode, combined output)."""
    path = os.path.join(OUT, f"{name}.txt")
    with open(path, "w") as f:
        f.write(script)
    env = dict(os.environ)
    env.update(ENV)
    p = subprocess.run([exe, path], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env,
                       timeout=600)
    return p.returncode, p.stdout
