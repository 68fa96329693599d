// Time-stepping kernels and launchers for 256x256 grids, double transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(double, 256)
