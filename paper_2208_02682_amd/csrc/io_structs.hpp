// Argument blocks of the float64 boundary transforms (host and device).
#pragma once

#include "fft_core.hpp"

namespace lm {

constexpr int IO_MAX = 8;

struct IoRowFwd {  // two physical fields -> two half-spectrum row fields
  const double* a[IO_MAX];
  const double* b[IO_MAX];  // may be null
  cplx<double>* oa[IO_MAX];
  cplx<double>* ob[IO_MAX];
};
struct IoColFwd {  // row-spectrum field -> normalised, truncated state
  const cplx<double>* src[IO_MAX];
  void* dst[IO_MAX];
  void* dst_lo[IO_MAX];  // float state: trailing words (value - leading word), or null
  int dst_f32[IO_MAX];
};
struct IoColInv {  // truncated state -> column-pass output
  const void* src[IO_MAX];
  const void* src_lo[IO_MAX];  // float state: trailing words added to the leading ones, or null
  int src_f32[IO_MAX];
  cplx<double>* dst[IO_MAX];
};
struct IoRowInv {  // two column-pass outputs -> two physical fields, scaled
  const cplx<double>* a[IO_MAX];
  const cplx<double>* b[IO_MAX];  // may be null
  double* oa[IO_MAX];
  double* ob[IO_MAX];
  double sa[IO_MAX];   // outputs are value * s + c
  double sb[IO_MAX];
  double ca[IO_MAX];
  double cb[IO_MAX];
};

}  // namespace lm
