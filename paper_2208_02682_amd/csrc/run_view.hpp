// Host-side view of one run: sizes, physics, stream and the sub-allocation of
// its single device slab.  Shared by the C ABI and the per-N launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include <type_traits>

#include "col_tile.hpp"
#include "fft_core.hpp"
#include "layout.hpp"
#include "step_args.hpp"

namespace lm {

constexpr size_t SLAB_ALIGN = 256;
inline size_t slab_up(size_t x) { return (x + SLAB_ALIGN - 1) / SLAB_ALIGN * SLAB_ALIGN; }

// float64 output planes of a closed interval: S2 mean h, zeta, xi_x, xi_y;
// S1 mean h, zeta, eta_x, eta_y; Eulerian h, zeta; the strategy-1 remap
// (mean h, zeta at mean positions, displacement x, y)
constexpr int NOUT = 14;
constexpr int OUT_REMAP = 10;
constexpr int OUT_MOM = 14;  // momentum 1-form mean x, y (planes 14, 15), when requested

// byte offsets of every buffer inside the slab
struct Layout {
  size_t Yr, Yl, Yd, Ar, Ad, Ys0, Ys1, IC, RS, uvhz, tw64, twT, out, phys, ioC, flag, resid, total;
};

// mom: also room for the strategy-2 mean of the momentum 1-form (its state,
// intermediates, row spectra and two output planes come last); gen: also the
// row spectra of the two averaged fields (Eulerian means of fields other than
// h and zeta)
inline Layout make_layout(const Dims& d, bool fp32, bool mom, bool gen) {
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
  const int nsf = mom ? NSF_R : SF_GMX, nic = mom ? NIC : IC_GMX;
  const int nrs = gen ? NRS : (mom ? RS_GMY + 1 : RS_GMX);
  L.Yr = take(nsf * sp * cT);
  // float state is carried in two words (leading in Yr, trailing here)
  L.Yl = take(fp32 ? nsf * sp * cT : 0);
  L.Yd = take(NSF_D * sp * cD);
  L.Ar = take(nsf * sp * cT);
  L.Ad = take(NSF_D * sp * cD);
  L.Ys0 = take(3 * sp * cT);
  L.Ys1 = take(3 * sp * cT);
  L.IC = take(nic * rf * cT);
  L.RS = take(nrs * rf * cT);
  L.uvhz = take(nn * 4 * (fp32 ? sizeof(float) : sizeof(double)));
  L.tw64 = take((size_t)d.N * cD);
  L.twT = take((size_t)d.N * cT);
  L.out = take((mom ? NOUT + 2 : NOUT) * nn * sizeof(double));
  L.phys = take(3 * nn * sizeof(double));
  L.ioC = take(10 * rf * cD);
  L.flag = take(sizeof(int));
  L.resid = take(sizeof(unsigned long long));
  L.total = o;
  return L;
}

// Launch schedule of the time-stepping kernels of one (N, precision): the
// column tile width (col_tile_of) and the block order (xcd_split).  Neither
// changes what a row or a column computes, or in which order.
struct Sched {
  int tile = 0;     // -1: half the default column tile width, 0: default, +1: twice
  int remap = 1;    // 1: XCD-aware block order, 0: hardware order
  int streams = 1;  // 1: the passes of a stage in order on the run's stream; 2: the
                    // stage's dependency graph on two streams (single runs only)
};

// Waits for a stream when it leaves scope, on every path out of a call: no
// copy or kernel the call enqueued can still touch a caller's buffer, a stack
// variable of the call, or memory released after the call returned.  (The
// wait's own status is not reported: an error path already has one.)
struct StreamDrain {
  hipStream_t s;
  ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

struct RunView {
  Dims d;
  Phys ph;
  hipStream_t stream;
  bool fp32;
  bool cubic;        // cubic strategy-2 gathers (else bilinear)
  bool mom;          // strategy-2 mean of the momentum 1-form as well
  Layout L;
  char* slab;
  int64_t n, n_tau;  // steps since set_state; step index at the interval start
  int ys_cur;        // which stage-value buffer holds the current stage input
  Sched sched;       // launch schedule used by the next launches
  hipStream_t aux = nullptr;  // second stream of the two-stream schedule
  hipEvent_t ev[4] = {};      // its fork, rows_dyn, rows_rhs and join events
  void* at(size_t off) const { return slab + off; }
};

template <typename T>
StepPtrs<T> step_ptrs(RunView& r) {
  StepPtrs<T> P;
  P.Yr = (cplx<T>*)r.at(r.L.Yr);
  P.Yl = std::is_same<T, float>::value ? (cplx<T>*)r.at(r.L.Yl) : nullptr;
  P.Yd = (cplx<double>*)r.at(r.L.Yd);
  P.Ar = (cplx<T>*)r.at(r.L.Ar);
  P.Ad = (cplx<double>*)r.at(r.L.Ad);
  P.IC = (cplx<T>*)r.at(r.L.IC);
  P.RS = (cplx<T>*)r.at(r.L.RS);
  P.uvhz = (P4<T>*)r.at(r.L.uvhz);
  P.tw = (const cplx<T>*)r.at(std::is_same<T, double>::value ? r.L.tw64 : r.L.twT);
  return P;
}

template <typename T>
RunDesc<T> run_desc(RunView& r, const long long* counter) {
  RunDesc<T> D;
  D.P = step_ptrs<T>(r);
  D.ph = r.ph;
  D.Ys0 = (cplx<T>*)r.at(r.L.Ys0);
  D.Ys1 = (cplx<T>*)r.at(r.L.Ys1);
  D.counter = counter;
  D.n_tau = r.n_tau;
  return D;
}

}  // namespace lm
