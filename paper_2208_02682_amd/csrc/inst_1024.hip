// Dispatchers and float64 boundary kernels for 1024x1024 grids (the
// time-stepping kernels are in inst_1024_f32.hip and inst_1024_f64.hip).
#include "launch_impl.hpp"

LM_INSTANTIATE(1024)
