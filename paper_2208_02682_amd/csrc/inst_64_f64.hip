// Time-stepping kernels and launchers for 64x64 grids, double transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(double, 64)
