// Time-stepping kernels and launchers for 1024x1024 grids, float transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(float, 1024)
