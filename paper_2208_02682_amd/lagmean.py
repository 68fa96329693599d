"""ctypes binding of liblagmean.so (include/lagmean.h); argument marshalling only.

Every computation happens in the HIP library.  Arrays may be NumPy float64
arrays (host) or device arrays: the library's own DeviceArray, or torch CUDA
float64 tensors when torch's HIP runtime is bound (LAGMEAN_HIP_RUNTIME=torch).
Loading the library fails loudly when it has not been built.
"""

from __future__ import annotations

import ctypes
import json
import os
from typing import Dict, List, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblagmean.so")

LM_OK = 0
STATUS = {0: "LM_OK", -1: "LM_E_ARG", -2: "LM_E_STATE", -3: "LM_E_OOM", -4: "LM_E_HIP",
          -5: "LM_E_NONFINITE", -6: "LM_E_UNSUPPORTED", -7: "LM_E_BUDGET"}
LM_FP64, LM_FP32_MIXED = 0, 1
(LM_K_S2_MEAN, LM_K_S2_XI_X, LM_K_S2_XI_Y, LM_K_S1_MEAN, LM_K_S1_ETA_X, LM_K_S1_ETA_Y, LM_K_EULER_MEAN,
 LM_K_S1_REMAP_MEAN, LM_K_S1_REMAP_XI_X, LM_K_S1_REMAP_XI_Y, LM_K_S2_MOM_X, LM_K_S2_MOM_Y) = range(12)
LM_F_H, LM_F_ZETA, LM_F_MOMENTUM, LM_F_U, LM_F_V, LM_F_Q = 1, 2, 4, 8, 16, 32
FIELD_BITS = {"h": LM_F_H, "zeta": LM_F_ZETA, "u": LM_F_U, "v": LM_F_V, "q": LM_F_Q}
LM_DYNAMIC, LM_KINEMATIC_PLANEWAVE = 0, 1
LM_STATIC_MAX_MEMBERS = 256  # members lm_batch_step_static accepts
LM_FIELD_H, LM_FIELD_ZETA = 0, 1
PEEK = {"u": 0, "v": 1, "h": 2, "gbar:h": 3, "gbar:zeta": 4, "gtil:h": 5, "gtil:zeta": 6,
        "E:h": 7, "E:zeta": 8, "xi_x": 9, "xi_y": 10, "P_x": 11, "P_y": 12}
# output names (the oracle's naming) -> (field, kind)
OUTPUTS = {
    "S2_mean:h": (LM_FIELD_H, LM_K_S2_MEAN), "S2_mean:zeta": (LM_FIELD_ZETA, LM_K_S2_MEAN),
    "S2_xi_x": (0, LM_K_S2_XI_X), "S2_xi_y": (0, LM_K_S2_XI_Y),
    "S1_mean:h": (LM_FIELD_H, LM_K_S1_MEAN), "S1_mean:zeta": (LM_FIELD_ZETA, LM_K_S1_MEAN),
    "S1_eta_x": (0, LM_K_S1_ETA_X), "S1_eta_y": (0, LM_K_S1_ETA_Y),
    "E_mean:h": (LM_FIELD_H, LM_K_EULER_MEAN), "E_mean:zeta": (LM_FIELD_ZETA, LM_K_EULER_MEAN),
}
# strategy-2 mean of the momentum 1-form (runs made with momentum=True)
MOMENTUM_OUTPUTS = {"S2_mom_x": (0, LM_K_S2_MOM_X), "S2_mom_y": (0, LM_K_S2_MOM_Y)}
# outputs of lm_remap_s1 (strategy 1 at Lagrangian-mean positions)
REMAP_OUTPUTS = {
    "S1R_mean:h": (LM_FIELD_H, LM_K_S1_REMAP_MEAN), "S1R_mean:zeta": (LM_FIELD_ZETA, LM_K_S1_REMAP_MEAN),
    "S1R_xi_x": (0, LM_K_S1_REMAP_XI_X), "S1R_xi_y": (0, LM_K_S1_REMAP_XI_Y),
}


class LagMeanError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("f", ctypes.c_double), ("g", ctypes.c_double), ("H", ctypes.c_double),
                ("dt", ctypes.c_double), ("nu8", ctypes.c_double),
                ("avg_fields", ctypes.c_uint32), ("strategies", ctypes.c_uint32),
                ("interp", ctypes.c_int32), ("mode", ctypes.c_int32), ("kin", ctypes.c_double * 8)]


class E2DConfig(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dt", ctypes.c_double), ("U0", ctypes.c_double), ("V0", ctypes.c_double),
                ("interp", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    """lm_schedule: column tile width (-1, 0, +1), XCD-aware block order (0, 1) and
    streams (1: the passes of a stage in order, 2: the stage's dependency graph on
    two streams)."""
    _fields_ = [("col_tile", ctypes.c_int32), ("xcd_order", ctypes.c_int32), ("streams", ctypes.c_int32)]

    def key(self) -> Tuple[int, int, int]:
        return (int(self.col_tile), int(self.xcd_order), int(self.streams))


E2D_OUTPUTS = {"zeta": 0, "PS_mean": 1, "PS_eta_x": 2, "PS_eta_y": 3, "SL_mean": 4, "SL_eta_x": 5, "SL_eta_y": 6}

_lib: Optional[ctypes.CDLL] = None


# Which HIP runtime the library binds (one per process).  Default ("own"): the
# runtime it was built with, loaded through its own dependency; the process must
# then not use torch's GPU functions.  "torch": PyTorch is imported first, and
# the library binds the runtime torch ships (an older one than the library is
# built with), so that torch CUDA tensors and streams can be passed in.
OWN_RUNTIME_ENV = "LAGMEAN_HIP_RUNTIME"


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2208_02682_amd.build`")
    # One HIP runtime per process.  PyTorch ships its own libamdhip64 (same
    # soname); loaded first, it is the runtime the library binds to, and loaded
    # after the library it would bring a second runtime that does not see the
    # GPU.  So torch is imported first only when its runtime is asked for.
    mode = os.environ.get(OWN_RUNTIME_ENV, "own")
    if mode not in ("own", "torch"):
        raise ValueError(f"{OWN_RUNTIME_ENV} must be 'own' or 'torch', not {mode!r}")
    if mode == "torch":
        import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lm_query_footprint": [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)],
        "lm_create": [ctypes.POINTER(Config), P, ctypes.POINTER(P)],
        "lm_set_state": [P, P, P, P, ctypes.c_int],
        "lm_get_state": [P, P, P, P, ctypes.c_int],
        "lm_begin_interval": [P],
        "lm_step": [P, ctypes.c_int32],
        "lm_step_profiled": [P, ctypes.c_int32, D],
        "lm_end_interval": [P, D],
        "lm_read_mean": [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int],
        "lm_remap_s1": [P, ctypes.c_int32, D],
        "lm_peek": [P, ctypes.c_int32, P, ctypes.c_int],
        "lm_counters": [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
        "lm_destroy": [P],
        "lm_hip_versions": [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
        "lm_device_alloc": [ctypes.c_size_t, ctypes.POINTER(P)],
        "lm_device_free": [P],
        "lm_memcpy": [P, P, ctypes.c_size_t, ctypes.c_int32],
        "lm_device_synchronize": [],
        "lm_copy_bandwidth": [ctypes.c_size_t, ctypes.c_int32, D],
        "lm_step_timed": [P, ctypes.c_int32, D],
        "lm_checkpoint_size": [P, ctypes.POINTER(ctypes.c_size_t)],
        "lm_save": [P, P, ctypes.c_size_t, ctypes.c_int],
        "lm_restore": [P, P, ctypes.c_size_t, ctypes.c_int],
        "lm_batch_create": [P, ctypes.POINTER(P)],
        "lm_batch_add": [P, P, ctypes.c_int32],
        "lm_batch_remove": [P, P],
        "lm_batch_step": [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
        "lm_batch_step_static": [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
        "lm_batch_remaining": [P, P, ctypes.POINTER(ctypes.c_int32)],
        "lm_batch_destroy": [P],
        "lm_schedule_candidates": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Schedule), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)],
        "lm_set_schedule": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Schedule)],
        "lm_get_schedule": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Schedule)],
        "lm_autotune": [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Schedule), D, ctypes.c_int32,
                        ctypes.POINTER(ctypes.c_int32)],
        "lm_set_batch_schedule": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Schedule)],
        "lm_get_batch_schedule": [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Schedule)],
        "lm_batch_autotune": [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
        "lm_e2d_create": [ctypes.POINTER(E2DConfig), P, ctypes.POINTER(P)],
        "lm_e2d_set_vorticity": [P, P, ctypes.c_int],
        "lm_e2d_begin_interval": [P],
        "lm_e2d_step": [P, ctypes.c_int32],
        "lm_e2d_step_profiled": [P, ctypes.c_int32, D, D],
        "lm_e2d_end_interval": [P, D],
        "lm_e2d_read": [P, ctypes.c_int32, P, ctypes.c_int],
        "lm_e2d_destroy": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.lm_status_str.argtypes = [ctypes.c_int]
    lib.lm_status_str.restype = ctypes.c_char_p
    lib.lm_last_error.argtypes = []
    lib.lm_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != LM_OK:
        msg = load_library().lm_last_error().decode()
        raise LagMeanError(status, msg)


LM_INTERP = {"bilinear": 0, "cubic": 1}


def make_config(n: int, *, precision: str = "fp64", f: float = 1.0, g: float = 1.0, H: float = 1.0,
                dt: float, nu8: float = 0.0, interp: str = "bilinear", momentum: bool = False,
                fields: Tuple[str, str] = ("h", "zeta"), kinematic: Optional[dict] = None) -> Config:
    """fields: the two averaged scalar fields (names of FIELD_BITS; output slot 0
    is the one with the lower bit).  kinematic: a prescribed flow instead of
    the dynamics, {"kx", "ky", "A", "omega" (0: dispersion), "phase", "U0", "V0"}."""
    prec = {"fp64": LM_FP64, "fp32": LM_FP32_MIXED}[precision]
    if len(fields) != 2 or len(set(fields)) != 2:
        raise ValueError("two distinct averaged fields")
    mask = FIELD_BITS[fields[0]] | FIELD_BITS[fields[1]]
    if momentum:
        mask |= LM_F_MOMENTUM
    cfg = Config(n=n, precision=prec, f=f, g=g, H=H, dt=dt, nu8=nu8, avg_fields=mask, strategies=0,
                 interp=LM_INTERP[interp], mode=LM_DYNAMIC)
    if kinematic is not None:
        cfg.mode = LM_KINEMATIC_PLANEWAVE
        for i, key in enumerate(("kx", "ky", "A", "omega", "phase", "U0", "V0")):
            cfg.kin[i] = float(kinematic.get(key, 0.0))
    return cfg


def field_slots(cfg: Config) -> Tuple[str, str]:
    """Names of the fields in output slots 0 and 1 of a configuration."""
    mask = int(cfg.avg_fields) & ~LM_F_MOMENTUM or (LM_F_H | LM_F_ZETA)
    names = [n for n, b in sorted(FIELD_BITS.items(), key=lambda kv: kv[1]) if mask & b]
    return names[0], names[1]


PRECISIONS = {"fp64": LM_FP64, "fp32": LM_FP32_MIXED}


def schedule_candidates(n: int, precision: str) -> List[Tuple[int, int, int]]:
    """Usable launch schedules (col_tile, xcd_order, streams) of single runs of
    (n, precision), the default first."""
    lib = load_library()
    buf = (Schedule * 16)()
    cnt = ctypes.c_int32(0)
    _check(lib.lm_schedule_candidates(n, PRECISIONS[precision], buf, len(buf), ctypes.byref(cnt)))
    return [buf[i].key() for i in range(cnt.value)]


def set_schedule(n: int, precision: str, col_tile: int, xcd_order: int, streams: int = 1,
                 batched: bool = False) -> None:
    """Install a schedule in the single-run table (or the batched launches' table)."""
    s = Schedule(col_tile=col_tile, xcd_order=xcd_order, streams=streams)
    lib = load_library()
    fn = lib.lm_set_batch_schedule if batched else lib.lm_set_schedule
    _check(fn(n, PRECISIONS[precision], ctypes.byref(s)))


def get_schedule(n: int, precision: str, batched: bool = False) -> Tuple[int, int, int]:
    s = Schedule()
    lib = load_library()
    fn = lib.lm_get_batch_schedule if batched else lib.lm_get_schedule
    _check(fn(n, PRECISIONS[precision], ctypes.byref(s)))
    return s.key()


def save_schedules(path: str, arch: str, tuned: List[dict]) -> None:
    """Write autotuning results as JSON: arch (the device's architecture name)
    and one entry per (context, n, precision) with the chosen schedule and, when
    measured, the per-step times of every candidate (Run.autotune's records;
    context "batched" for Batch.autotune's)."""
    entries = []
    for t in tuned:
        best = tuple(t["best"]) + (1,) * (3 - len(t["best"]))
        entries.append({"context": t.get("context", "single"), "n": int(t["n"]), "precision": t["precision"],
                        "col_tile": int(best[0]), "xcd_order": int(best[1]), "streams": int(best[2]),
                        "ms_per_step": {",".join(str(x) for x in k): float(v) for k, v in t.get("ms", {}).items()}})
    with open(path, "w") as f:
        json.dump({"format": 1, "arch": arch, "entries": entries}, f, indent=1)


def load_schedules(path: str, arch: Optional[str] = None) -> int:
    """Apply the schedules of a JSON cache written by save_schedules (only if
    its arch matches, when arch is given); returns the number applied."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != 1:
        raise ValueError(f"{path}: unknown schedule cache format")
    if arch is not None and doc.get("arch") != arch:
        return 0
    for e in doc["entries"]:
        set_schedule(int(e["n"]), e["precision"], int(e["col_tile"]), int(e["xcd_order"]), int(e.get("streams", 1)),
                     batched=e.get("context", "single") == "batched")
    return len(doc["entries"])


def hip_runtime() -> Dict[str, object]:
    """HIP versions the library was built with and runs on (lm_hip_versions),
    and the file of the HIP runtime the process has mapped."""
    lib = load_library()
    built, runtime = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib.lm_hip_versions(ctypes.byref(built), ctypes.byref(runtime)))
    files = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    files.add(line.split()[-1])
    except OSError:
        pass
    return {"built": int(built.value), "runtime": int(runtime.value), "runtime_files": sorted(files),
            "same": int(built.value) // 100000 == int(runtime.value) // 100000}


def footprint(cfg: Config) -> int:
    out = ctypes.c_size_t(0)
    _check(load_library().lm_query_footprint(ctypes.byref(cfg), ctypes.byref(out)))
    return int(out.value)


class DeviceArray:
    """A float64 array in device memory allocated by the library (lm_device_alloc)."""

    def __init__(self, shape, host=None):
        self.lib = load_library()
        self.shape = tuple(int(x) for x in shape)
        self.nbytes = int(np.prod(self.shape)) * 8
        self.ptr = ctypes.c_void_p(0)
        _check(self.lib.lm_device_alloc(self.nbytes, ctypes.byref(self.ptr)))
        if host is not None:
            self.copy_from(host)

    @classmethod
    def from_host(cls, a) -> "DeviceArray":
        a = np.ascontiguousarray(a, dtype=np.float64)
        return cls(a.shape, a)

    def copy_from(self, a) -> None:
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != self.shape:
            raise ValueError(f"expected shape {self.shape}, got {a.shape}")
        _check(self.lib.lm_memcpy(self.ptr, a.ctypes.data_as(ctypes.c_void_p), self.nbytes, 0))

    def to_host(self) -> np.ndarray:
        out = np.empty(self.shape)
        _check(self.lib.lm_memcpy(out.ctypes.data_as(ctypes.c_void_p), self.ptr, self.nbytes, 1))
        return out

    def close(self) -> None:
        if self.ptr and self.ptr.value:
            _check(self.lib.lm_device_free(self.ptr))
            self.ptr = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_synchronize() -> None:
    _check(load_library().lm_device_synchronize())


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """GB/s of a plain device copy of nbytes (read + written), lm_copy_bandwidth."""
    g = ctypes.c_double(0.0)
    _check(load_library().lm_copy_bandwidth(int(nbytes), int(reps), ctypes.byref(g)))
    return g.value


def _is_device(a) -> bool:
    return isinstance(a, DeviceArray) or (hasattr(a, "is_cuda") and bool(a.is_cuda))


def _ptr(a):
    if isinstance(a, DeviceArray):
        return a.ptr
    if _is_device(a):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _host_in(a, N):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (N, N):
        raise ValueError(f"expected an {N}x{N} array, got {a.shape}")
    return a


class Run:
    """One averaging run on the GPU (wraps lm_run)."""

    def __init__(self, cfg: Config, stream: int = 0):
        self.lib = load_library()
        self.cfg = cfg
        self.N = cfg.n
        self.h = ctypes.c_void_p(0)
        _check(self.lib.lm_create(ctypes.byref(cfg), ctypes.c_void_p(stream), ctypes.byref(self.h)))

    # -- lifetime
    def close(self) -> None:
        if self.h and self.h.value:
            _check(self.lib.lm_destroy(self.h))
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- state
    def set_state(self, u, v, h) -> None:
        if _is_device(u):
            for a in (u, v, h):
                if isinstance(a, DeviceArray):
                    ok = a.shape == (self.N, self.N)
                else:
                    ok = str(a.dtype) == "torch.float64" and a.is_contiguous() and tuple(a.shape) == (self.N, self.N)
                if not ok:
                    raise ValueError("device inputs must be contiguous float64 N x N arrays")
            _check(self.lib.lm_set_state(self.h, _ptr(u), _ptr(v), _ptr(h), 1))
        else:
            u, v, h = (_host_in(a, self.N) for a in (u, v, h))
            _check(self.lib.lm_set_state(self.h, _ptr(u), _ptr(v), _ptr(h), 0))

    def get_state(self):
        out = [np.empty((self.N, self.N)) for _ in range(3)]
        _check(self.lib.lm_get_state(self.h, *(_ptr(a) for a in out), 0))
        return tuple(out)

    # -- averaging
    def begin_interval(self) -> None:
        _check(self.lib.lm_begin_interval(self.h))

    def step(self, nsteps: int = 1) -> None:
        _check(self.lib.lm_step(self.h, int(nsteps)))

    def step_timed(self, nsteps: int) -> float:
        """Milliseconds of nsteps steps between HIP events on the run's stream (lm_step_timed)."""
        ms = ctypes.c_double(0.0)
        _check(self.lib.lm_step_timed(self.h, int(nsteps), ctypes.byref(ms)))
        return ms.value

    def step_profiled(self, nsteps: int):
        """Average milliseconds of (rows_dyn, rows_rhs, columns) over nsteps steps."""
        ms = (ctypes.c_double * 3)()
        _check(self.lib.lm_step_profiled(self.h, int(nsteps), ms))
        return list(ms)

    def end_interval(self) -> float:
        T = ctypes.c_double(0.0)
        _check(self.lib.lm_end_interval(self.h, ctypes.byref(T)))
        return T.value

    def read_mean(self, field: int, kind: int, out=None):
        if out is None:
            out = np.empty((self.N, self.N))
        _check(self.lib.lm_read_mean(self.h, field, kind, _ptr(out), 1 if _is_device(out) else 0))
        return out

    def outputs(self) -> Dict[str, np.ndarray]:
        """The interval's outputs, named as the oracle's (the default fields h and
        zeta); runs averaging other fields use field_outputs."""
        return {name: self.read_mean(fk[0], fk[1]) for name, fk in OUTPUTS.items()}

    def field_outputs(self) -> Dict[str, np.ndarray]:
        """The interval's outputs named by the run's averaged fields, as the
        oracle names them (e.g. "S2_mean:u", "S1_mean:q", "E_mean:v", "S2_xi_x")."""
        slots = field_slots(self.cfg)
        out = {}
        for name, (fld, kind) in OUTPUTS.items():
            if ":" in name:
                base = name.split(":")[0]
                out[f"{base}:{slots[fld]}"] = self.read_mean(fld, kind)
            else:
                out[name] = self.read_mean(fld, kind)
        return out

    def remap_s1(self, max_extent: int = 64) -> float:
        """Strategy 1 at Lagrangian-mean positions (lm_remap_s1); returns the
        largest inversion residual in grid spacings (inf if a point is not covered)."""
        res = ctypes.c_double(0.0)
        _check(self.lib.lm_remap_s1(self.h, int(max_extent), ctypes.byref(res)))
        return res.value

    def momentum_outputs(self) -> Dict[str, np.ndarray]:
        return {name: self.read_mean(fk[0], fk[1]) for name, fk in MOMENTUM_OUTPUTS.items()}

    def remap_outputs(self) -> Dict[str, np.ndarray]:
        return {name: self.read_mean(fk[0], fk[1]) for name, fk in REMAP_OUTPUTS.items()}

    def autotune(self, steps: int = 8, reps: int = 3) -> dict:
        """Time every launch schedule of this run's (N, precision) on a copy of
        its state (lm_autotune; the run itself is left as it was) and make the
        fastest the schedule of that (N, precision).  Returns {"n", "precision",
        "best": (col_tile, xcd_order), "ms": {schedule: ms per step}}."""
        cand = schedule_candidates(self.N, "fp32" if self.cfg.precision == LM_FP32_MIXED else "fp64")
        ms = (ctypes.c_double * len(cand))()
        best = Schedule()
        cnt = ctypes.c_int32(0)
        _check(self.lib.lm_autotune(self.h, int(steps), int(reps), ctypes.byref(best), ms, len(cand),
                                    ctypes.byref(cnt)))
        return {"n": self.N, "precision": "fp32" if self.cfg.precision == LM_FP32_MIXED else "fp64",
                "best": best.key(), "ms": {cand[i]: ms[i] for i in range(cnt.value)}}

    def peek(self, which: str):
        out = np.empty((self.N, self.N))
        _check(self.lib.lm_peek(self.h, PEEK[which], _ptr(out), 0))
        return out

    def save(self) -> np.ndarray:
        """A checkpoint of the run between steps (lm_save), as bytes on the host."""
        n = ctypes.c_size_t(0)
        _check(self.lib.lm_checkpoint_size(self.h, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        _check(self.lib.lm_save(self.h, buf.ctypes.data_as(ctypes.c_void_p), n.value, 0))
        return buf

    def restore(self, blob) -> None:
        """Continue from a checkpoint taken with lm_save of a run of the same configuration."""
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        _check(self.lib.lm_restore(self.h, b.ctypes.data_as(ctypes.c_void_p), b.size, 0))

    def counters(self):
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(self.lib.lm_counters(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


class Batch:
    """Runs of any N and precision advanced together (wraps lm_batch).

    A member needs a state and an open interval; it is advanced by up to its
    step budget.  While a member, a run is driven only through the batch."""

    def __init__(self, stream: int = 0):
        self.lib = load_library()
        self.h = ctypes.c_void_p(0)
        self.members = []
        _check(self.lib.lm_batch_create(ctypes.c_void_p(stream), ctypes.byref(self.h)))

    def add(self, run: Run, steps: int) -> None:
        _check(self.lib.lm_batch_add(self.h, run.h, int(steps)))
        self.members.append(run)

    def remove(self, run: Run) -> None:
        _check(self.lib.lm_batch_remove(self.h, run.h))
        self.members.remove(run)

    def step(self, max_steps: int) -> int:
        """Advance every member by min(max_steps, its budget); returns how many
        members still have budget left."""
        active = ctypes.c_int32(0)
        _check(self.lib.lm_batch_step(self.h, int(max_steps), ctypes.byref(active)))
        return active.value

    def step_static(self, max_steps: int) -> int:
        """As step, through the allocation-free lm_batch_step_static."""
        active = ctypes.c_int32(0)
        _check(self.lib.lm_batch_step_static(self.h, int(max_steps), ctypes.byref(active)))
        return active.value

    def autotune(self, steps: int = 4, reps: int = 3) -> List[dict]:
        """Tune the batched launches' schedule of every (N, precision) among the
        members (lm_batch_autotune; members are left as they were).  Returns one
        record per (N, precision) with the chosen schedule (context "batched")."""
        n = ctypes.c_int32(0)
        _check(self.lib.lm_batch_autotune(self.h, int(steps), int(reps), ctypes.byref(n)))
        keys = sorted({(r.N, "fp32" if r.cfg.precision == LM_FP32_MIXED else "fp64") for r in self.members})
        return [{"context": "batched", "n": N, "precision": p, "best": get_schedule(N, p, batched=True)}
                for N, p in keys]

    def remaining(self, run: Run) -> int:
        r = ctypes.c_int32(0)
        _check(self.lib.lm_batch_remaining(self.h, run.h, ctypes.byref(r)))
        return r.value

    def close(self) -> None:
        if self.h and self.h.value:
            _check(self.lib.lm_batch_destroy(self.h))
            self.h = ctypes.c_void_p(0)
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Euler2D:
    """Two-dimensional incompressible flow with strategy 1 pseudospectral and
    semi-Lagrangian (wraps lm_e2d, float64)."""

    def __init__(self, n: int, dt: float, *, U0: float = 0.0, V0: float = 0.0, interp: str = "bilinear",
                 stream: int = 0):
        self.lib = load_library()
        self.N = n
        self.h = ctypes.c_void_p(0)
        cfg = E2DConfig(n=n, dt=dt, U0=U0, V0=V0, interp=LM_INTERP[interp])
        _check(self.lib.lm_e2d_create(ctypes.byref(cfg), ctypes.c_void_p(stream), ctypes.byref(self.h)))

    def close(self) -> None:
        if self.h and self.h.value:
            _check(self.lib.lm_e2d_destroy(self.h))
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_vorticity(self, zeta) -> None:
        dev = _is_device(zeta)
        a = zeta if dev else _host_in(zeta, self.N)
        _check(self.lib.lm_e2d_set_vorticity(self.h, _ptr(a), 1 if dev else 0))

    def begin_interval(self) -> None:
        _check(self.lib.lm_e2d_begin_interval(self.h))

    def step(self, nsteps: int = 1) -> None:
        _check(self.lib.lm_e2d_step(self.h, int(nsteps)))

    def step_timed(self, nsteps: int) -> float:
        """Milliseconds of nsteps steps between HIP events on the run's stream (lm_step_timed)."""
        ms = ctypes.c_double(0.0)
        _check(self.lib.lm_step_timed(self.h, int(nsteps), ctypes.byref(ms)))
        return ms.value

    def step_profiled(self, nsteps: int):
        """(average step, average semi-Lagrangian kernel) in milliseconds."""
        a, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(self.lib.lm_e2d_step_profiled(self.h, int(nsteps), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def end_interval(self) -> float:
        T = ctypes.c_double(0.0)
        _check(self.lib.lm_e2d_end_interval(self.h, ctypes.byref(T)))
        return T.value

    def read(self, kind: str, out=None):
        if out is None:
            out = np.empty((self.N, self.N))
        _check(self.lib.lm_e2d_read(self.h, E2D_OUTPUTS[kind], _ptr(out), 1 if _is_device(out) else 0))
        return out

    def outputs(self) -> Dict[str, np.ndarray]:
        return {k: self.read(k) for k in E2D_OUTPUTS}
