// Kernels and launchers for 64x64 grids.
#include "launch_impl.hpp"

LM_INSTANTIATE(64)
