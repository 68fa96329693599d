// Kernels and launchers for 512x512 grids.
#include "launch_impl.hpp"

LM_INSTANTIATE(512)
