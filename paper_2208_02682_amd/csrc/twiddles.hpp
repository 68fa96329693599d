// Host side: the twiddle table of an N-point transform in the stage-by-stage
// layout the device transforms read (fft_core.hpp).
#pragma once

#include <cmath>
#include <vector>

#include "fft_core.hpp"

namespace lm {

// One block per stage of the plan of n (radix R after sub-transforms of length
// Ns): entry (r - 1) Ns + k = exp(-2 pi i m / n), m = r k n / (Ns R), for
// r = 1..R-1, k < Ns; computed in long double.  The table fills the first
// tw_len(n) of n slots (the rest is zero).
template <typename T>
std::vector<cplx<T>> stage_twiddles(int n) {
  const int e = fft_E_of(n);
  const Radices p = plan_of(n, e);
  const int R[3] = {p.R2, p.R3, p.R4};
  std::vector<cplx<T>> tw((size_t)n, cplx<T>{T(0), T(0)});
  int ns = e;
  for (int s = 0; s < 3; ++s) {
    const int off = tw_offset(n, e, s);
    for (int r = 1; r < R[s]; ++r)
      for (int k = 0; k < ns; ++k) {
        const long long m = (long long)r * k * (n / (ns * R[s]));
        const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)n;
        tw[(size_t)off + (size_t)(r - 1) * ns + k] = {(T)cosl(a), (T)sinl(a)};
      }
    ns *= R[s];
  }
  return tw;
}

}  // namespace lm
