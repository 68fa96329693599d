"""Workload table: grid size, physics, time step, averaging interval and seeds.

Every number here is a configuration choice, not part of the method:

* ``nu8_rule``: eighth-order hyperviscosity coefficient nu8 = 0.1 / (dt K^8) with
  K = floor((N-1)/3), i.e. the hyperviscous decay over one step at the
  dealiasing cutoff on an axis is 0.1.
* ``averaging_steps``: the averaging interval is ``periods`` periods of the
  slowest wave in the band, omega_lo = sqrt(f^2 + g H k_lo^2), rounded to a
  whole number of steps (the paper averages over about 3.6 wave periods in its
  section 4.2.1).
* the "R2" scaling of the batched and served workloads multiplies the
  wavenumbers of the 64^2 recipe by N/64 and sets dt = 0.64 / N, so that the
  flow is the same in grid units.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from .fields import turbulence_plus_waves


def nu8_rule(N: int, dt: float) -> float:
    K = (N - 1) // 3
    return 0.1 / (dt * float(K) ** 8)


def averaging_steps(k_lo: float, dt: float, periods: float = 3.6,
                    f: float = 1.0, g: float = 1.0, H: float = 1.0) -> int:
    omega_lo = math.sqrt(f * f + g * H * k_lo * k_lo)
    return int(round(periods * 2.0 * math.pi / omega_lo / dt))


@dataclass(frozen=True)
class Workload:
    name: str
    N: int
    precision: str            # "fp64" or "fp32" (FP32 transforms, FP64 xi/P state)
    k0: float
    Ro: float
    k_lo: float
    k_hi: float
    ratio: float
    seed_vortex: int
    seed_wave: int
    dt: float
    steps_per_interval: int
    n_intervals: int
    nu8: float
    f: float = 1.0
    g: float = 1.0
    H: float = 1.0

    @property
    def T(self) -> float:
        return self.steps_per_interval * self.dt

    @property
    def total_steps(self) -> int:
        return self.steps_per_interval * self.n_intervals

    def initial_state(self):
        return turbulence_plus_waves(
            self.N, k0=self.k0, Ro=self.Ro, k_lo=self.k_lo, k_hi=self.k_hi,
            ratio=self.ratio, seed_vortex=self.seed_vortex, seed_wave=self.seed_wave,
            f=self.f, g=self.g, H=self.H)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def _make(name, N, precision, k0, Ro, k_lo, k_hi, ratio, seeds, dt, n_intervals,
          periods=3.6):
    return Workload(name=name, N=N, precision=precision, k0=k0, Ro=Ro, k_lo=k_lo,
                    k_hi=k_hi, ratio=ratio, seed_vortex=seeds[0], seed_wave=seeds[1],
                    dt=dt, steps_per_interval=averaging_steps(k_lo, dt, periods),
                    n_intervals=n_intervals, nu8=nu8_rule(N, dt))


# 64^2 FP64 single run: spectrum k^4 exp(-(k/6)^2), Ro 0.05, waves |k| in [2, 4].
CFG_SMALL = _make("sw64_fp64", 64, "fp64", 6.0, 0.05, 2.0, 4.0, 1.0, (0, 1), 0.01, 1)
# 256^2 FP64, spectrum peak k = 12 (k0 = 12/sqrt 2), waves [4, 8], 4 intervals.
CFG_MEDIUM = _make("sw256_fp64", 256, "fp64", 12.0 / math.sqrt(2.0), 0.05, 4.0, 8.0, 1.0,
                   (2, 3), 0.0025, 4)
# 1024^2 FP32 transforms with FP64 displacement accumulators, peak k = 32, Ro 0.1.
CFG_LARGE = _make("sw1024_fp32", 1024, "fp32", 32.0 / math.sqrt(2.0), 0.1, 8.0, 16.0, 1.0,
                  (4, 5), 6e-4, 2)
# The 1024^2 recipe scaled to 256^2 (wavenumbers / 4, dt * 4): the full cross-run.
CFG_LARGE_AT_256 = _make("sw1024recipe_at256_fp32", 256, "fp32", 8.0 / math.sqrt(2.0), 0.1,
                         2.0, 4.0, 1.0, (4, 5), 2.4e-3, 2)

WORKLOADS = {w.name: w for w in (CFG_SMALL, CFG_MEDIUM, CFG_LARGE, CFG_LARGE_AT_256)}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def scaled_run(N: int, *, Ro: float, ratio: float, periods: float, seeds, precision="fp32",
               base_k0: float = 6.0, base_band=(2.0, 4.0)) -> Workload:
    """The 64^2 recipe scaled to N (R2 scaling)."""
    s = N / 64.0
    dt = 0.64 / N
    k_lo, k_hi = base_band[0] * s, base_band[1] * s
    return _make(f"run{N}", N, precision, base_k0 * s, Ro, k_lo, k_hi, ratio, seeds, dt, 1,
                 periods=periods)


def batch_workloads(count: int = 64, seed: int = 999, sizes=(128, 192, 256, 384, 512)):
    """Independent uneven runs: N uniform over ``sizes``, Ro ~ U[0.02, 0.2],
    energy ratio log-uniform in [0.25, 4], T uniform in [1, 8] wave periods."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        N = int(sizes[rng.integers(len(sizes))])
        Ro = float(rng.uniform(0.02, 0.2))
        ratio = float(np.exp(rng.uniform(np.log(0.25), np.log(4.0))))
        periods = float(rng.uniform(1.0, 8.0))
        out.append(scaled_run(N, Ro=Ro, ratio=ratio, periods=periods,
                              seeds=(1000 + 2 * i, 1001 + 2 * i)))
    return out


@dataclass
class Request:
    index: int
    arrival: float
    run: Workload = field(repr=False)


def serving_requests(rate: float = 20.0, duration: float = 300.0, seed: int = 7,
                     sizes=(128, 256, 512, 1024), probs=(0.4, 0.3, 0.2, 0.1)):
    """Poisson arrivals of averaging requests; request j uses field seeds
    (2000 + 2j, 2001 + 2j) and the 64^2 recipe scaled to its N."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    j = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        N = int(rng.choice(np.asarray(sizes), p=np.asarray(probs)))
        periods = float(rng.uniform(1.0, 8.0))
        run = scaled_run(N, Ro=0.05, ratio=1.0, periods=periods,
                         seeds=(2000 + 2 * j, 2001 + 2 * j))
        out.append(Request(j, t, run))
        j += 1
    return out
