// Time-stepping kernels and launchers for 192x192 grids, double transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(double, 192)
