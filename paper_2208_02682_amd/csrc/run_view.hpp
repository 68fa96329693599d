// Host-side view of one run: sizes, physics, stream and the sub-allocation of
// its single device slab.  Shared by the C ABI and the per-N launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fft_core.hpp"
#include "layout.hpp"

namespace lm {

constexpr size_t SLAB_ALIGN = 256;
inline size_t slab_up(size_t x) { return (x + SLAB_ALIGN - 1) / SLAB_ALIGN * SLAB_ALIGN; }

// byte offsets of every buffer inside the slab
struct Layout {
  size_t Yr, Yd, Ar, Ad, Ys0, Ys1, IC, RS, uvhz, tw64, twT, out, phys, ioC, flag, total;
};

inline Layout make_layout(const Dims& d, bool fp32) {
  const size_t cT = fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  const size_t cD = sizeof(cplx<double>);
  const size_t sp = d.spec_elems(), rf = d.rowfield_elems(), nn = (size_t)d.N * d.N;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += slab_up(bytes);
    return at;
  };
  L.Yr = take(NSF_R * sp * cT);
  L.Yd = take(NSF_D * sp * cD);
  L.Ar = take(NSF_R * sp * cT);
  L.Ad = take(NSF_D * sp * cD);
  L.Ys0 = take(3 * sp * cT);
  L.Ys1 = take(3 * sp * cT);
  L.IC = take(NIC * rf * cT);
  L.RS = take(NRS * rf * cT);
  L.uvhz = take(nn * 4 * (fp32 ? sizeof(float) : sizeof(double)));
  L.tw64 = take((size_t)d.N * cD);
  L.twT = take((size_t)d.N * cT);
  L.out = take(10 * nn * sizeof(double));
  L.phys = take(3 * nn * sizeof(double));
  L.ioC = take(10 * rf * cD);
  L.flag = take(sizeof(int));
  L.total = o;
  return L;
}

struct RunView {
  Dims d;
  Phys ph;
  hipStream_t stream;
  bool fp32;
  Layout L;
  char* slab;
  int64_t n, n_tau;  // steps since set_state; step index at the interval start
  int ys_cur;        // which stage-value buffer holds the current stage input
  void* at(size_t off) const { return slab + off; }
};

}  // namespace lm
