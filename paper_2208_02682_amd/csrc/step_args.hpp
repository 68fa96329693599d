// Argument blocks of the hot-path kernels (shared by host and device code).
#pragma once

#include "fft_core.hpp"
#include "layout.hpp"

namespace lm {

template <typename T>
struct alignas(4 * sizeof(T)) P4 {
  T u, v, h, z;
};

template <typename T>
struct StepPtrs {
  cplx<T>* Yr;        // [NSF_R][NKX][NKY] state, working precision
  cplx<T>* Yl;        // same shape: trailing words of compensated float state (unused in float64)
  cplx<double>* Yd;   // [NSF_D][NKX][NKY] state, float64
  cplx<T>* Ar;        // RK4 accumulators, same shapes
  cplx<double>* Ad;
  cplx<T>* IC;        // [NIC][N][NKXP] column-pass outputs
  cplx<T>* RS;        // [NRS][N][NKXP] row-pass outputs
  P4<T>* uvhz;        // [N][N] physical u, v, h, zeta
  const cplx<T>* tw;  // [N] exp(-2 pi i m / N)
};

// what a batched launch needs to know about one run
template <typename T>
struct RunDesc {
  StepPtrs<T> P;
  Phys ph;
  cplx<T>* Ys0;              // stage values of u, v, h (ping-pong buffers)
  cplx<T>* Ys1;
  const long long* counter;  // RK4 steps since the interval start
  long long n_tau;           // steps from the state's time origin to the interval start
};

}  // namespace lm
