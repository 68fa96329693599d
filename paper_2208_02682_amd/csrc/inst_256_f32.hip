// Time-stepping kernels and launchers for 256x256 grids, float transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(float, 256)
