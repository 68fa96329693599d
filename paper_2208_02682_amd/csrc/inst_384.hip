// Dispatchers and float64 boundary kernels for 384x384 grids (the
// time-stepping kernels are in inst_384_f32.hip and inst_384_f64.hip).
#include "launch_impl.hpp"

LM_INSTANTIATE(384)
