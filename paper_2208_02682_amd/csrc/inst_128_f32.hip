// Time-stepping kernels and launchers for 128x128 grids, float transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(float, 128)
