// Dispatchers and float64 boundary kernels for 128x128 grids (the
// time-stepping kernels are in inst_128_f32.hip and inst_128_f64.hip).
#include "launch_impl.hpp"

LM_INSTANTIATE(128)
