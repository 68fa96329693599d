// Dispatchers and float64 boundary kernels for 192x192 grids (the
// time-stepping kernels are in inst_192_f32.hip and inst_192_f64.hip).
#include "launch_impl.hpp"

LM_INSTANTIATE(192)
