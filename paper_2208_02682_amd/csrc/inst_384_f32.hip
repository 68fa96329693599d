// Time-stepping kernels and launchers for 384x384 grids, float transforms.
#include "launch_impl.hpp"

LM_INSTANTIATE_T(float, 384)
