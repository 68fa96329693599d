// Time-stepping kernels and launchers for 192x192 grids, float transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(float, 192)
