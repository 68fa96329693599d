// Kernels and launchers for 256x256 grids.
#include "launch_impl.hpp"

LM_INSTANTIATE(256)
