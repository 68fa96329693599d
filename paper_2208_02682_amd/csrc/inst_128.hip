// Kernels and launchers for 128x128 grids.
#include "launch_impl.hpp"

LM_INSTANTIATE(128)
