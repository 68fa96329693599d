"""MI355X-native Lagrangian means: rotating shallow water + the Lagrangian-mean
PDEs of Kafiabad & Vanneste ("Computing Lagrangian means"), both strategies,
advanced together in hand-written HIP kernels behind the C ABI of
include/lagmean.h.  This package is the thin Python binding (``lagmean``), the
build script (``build``) and the batch/serving drivers."""

from .lagmean import (LagMeanError, Run, Batch, Euler2D, Config, make_config, footprint, load_library, OUTPUTS, REMAP_OUTPUTS, PEEK,
                      LM_FIELD_H, LM_FIELD_ZETA, schedule_candidates, set_schedule, get_schedule, save_schedules,
                      load_schedules, hip_runtime, DeviceArray, device_synchronize, copy_bandwidth)

__all__ = ["LagMeanError", "Run", "Batch", "Euler2D", "Config", "make_config", "footprint", "load_library", "OUTPUTS", "REMAP_OUTPUTS", "PEEK",
           "LM_FIELD_H", "LM_FIELD_ZETA", "schedule_candidates", "set_schedule", "get_schedule", "save_schedules",
           "load_schedules", "hip_runtime", "DeviceArray", "device_synchronize", "copy_bandwidth"]
