// Dispatchers and float64 boundary kernels for 256x256 grids (the
// time-stepping kernels are in inst_256_f32.hip and inst_256_f64.hip).
#include "launch_impl.hpp"

LM_INSTANTIATE(256)
