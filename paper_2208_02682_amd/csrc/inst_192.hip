// Kernels and launchers for 192x192 grids.
#include "launch_impl.hpp"

LM_INSTANTIATE(192)
