// Time-stepping kernels and launchers for 1024x1024 grids, double transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(double, 1024)
