// Time-stepping kernels and launchers for 512x512 grids, double transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(double, 512)
