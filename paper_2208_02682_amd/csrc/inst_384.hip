// Kernels and launchers for 384x384 grids.
#include "launch_impl.hpp"

LM_INSTANTIATE(384)
