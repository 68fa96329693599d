// Time-stepping kernels and launchers for 64x64 grids, float transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(float, 64)
