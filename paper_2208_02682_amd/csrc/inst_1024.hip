// Kernels and launchers for 1024x1024 grids.
#include "launch_impl.hpp"

LM_INSTANTIATE(1024)
