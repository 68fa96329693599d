// Dispatchers and float64 boundary kernels for 64x64 grids (the
// time-stepping kernels are in inst_64_f32.hip and inst_64_f64.hip).
#include "launch_impl.hpp"

LM_INSTANTIATE(64)
