// Dispatchers and float64 boundary kernels for 512x512 grids (the
// time-stepping kernels are in inst_512_f32.hip and inst_512_f64.hip).
#include "launch_impl.hpp"

LM_INSTANTIATE(512)
