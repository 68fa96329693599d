// Time-stepping kernels and launchers for 128x128 grids, double transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(double, 128)
