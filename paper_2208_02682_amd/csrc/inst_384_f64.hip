// Time-stepping kernels and launchers for 384x384 grids, double transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(double, 384)
