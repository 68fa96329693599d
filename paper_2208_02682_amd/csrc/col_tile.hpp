// Column tiles of the column pass: how many spectral columns one block
// transforms.  Shared by the kernels and by the host code that checks launch
// schedules.
#pragma once

#include "fft_core.hpp"

namespace lm {

// column tile width: 8 columns (64-byte row segments in float32), or more when a
// transform needs fewer than 8 lanes, so that a block is at least one wavefront.
// W = -1 / +1: half / twice that width (the alternative launch schedules; the
// arithmetic of every column is the same whatever the width)
__host__ __device__ constexpr int col_tile_of(int n, int w) {
  const int base = (n / fft_E_of(n) >= 8) ? 8 : 64 / (n / fft_E_of(n));
  return w < 0 ? base / 2 : (w > 0 ? base * 2 : base);
}
__host__ __device__ constexpr int col_buf(int N) { return padded_len(N) | 1; }
// a width is usable when its block is whole wavefronts (at most 1024 threads)
// and its LDS fits in a CU's 160 KiB
__host__ __device__ constexpr bool col_tile_usable(int n, int w, int cplx_bytes) {
  const int threads = col_tile_of(n, w) * (n / fft_E_of(n));
  return col_tile_of(n, w) >= 1 && threads >= 64 && threads % 64 == 0 && threads <= 1024 &&
         (long long)col_tile_of(n, w) * col_buf(n) * cplx_bytes <= 160LL * 1024;
}

}  // namespace lm
