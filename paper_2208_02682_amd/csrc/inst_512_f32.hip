// Time-stepping kernels and launchers for 512x512 grids, float transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(float, 512)
