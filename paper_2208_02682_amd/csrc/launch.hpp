// Per-N launchers (explicitly instantiated in inst_<N>.hip so that the
// kernels of different grid sizes compile in parallel).
#pragma once

#include "io_structs.hpp"
#include "run_view.hpp"

namespace lm {

template <int N> void launch_steps(RunView& r, int nsteps);   // nsteps RK4 steps
template <int N> hipError_t launch_steps_profiled(RunView& r, int nsteps, double* ms);  // + kernel times
template <int N> void launch_prologue(RunView& r);            // column pass of the current state
// one RK4 step for nruns runs of one (N, precision, gather, momentum) group; desc: device array of RunDesc<T>
// ncg: column groups per run (col_groups of the group's runs)
template <int N> void launch_batch_step(hipStream_t st, const void* desc, int nruns, bool fp32, bool cubic, bool mom,
                                        int ncg, const Sched& sc);
void launch_batch_tick(hipStream_t st, long long* counters, int n);  // counters[i] += 1
template <int N> void launch_io_row_forward(RunView& r, const IoRowFwd& J, int count);
template <int N> void launch_io_col_forward(RunView& r, const IoColFwd& J, int count);
template <int N> void launch_io_col_inverse(RunView& r, const IoColInv& J, int count);
template <int N> void launch_io_row_inverse(RunView& r, const IoRowInv& J, int count);
void launch_nonfinite(RunView& r, const double* a, size_t n, int* flag);
// two-dimensional incompressible flow (float64): spectral multipliers, products,
// Heun stages and the semi-Lagrangian update (euler2d_kernels.hip)
void launch_e2d_spec(hipStream_t st, const Dims& d, const cplx<double>* Y, cplx<double>* S);
void launch_e2d_products(hipStream_t st, int nn, const double* PH, double* NL, double s);
void launch_e2d_stage(hipStream_t st, size_t sp, cplx<double>* Y, cplx<double>* Y1, cplx<double>* K1,
                      const cplx<double>* R, double dt, int stage);
void launch_e2d_sl(hipStream_t st, int N, const double* u, const double* v, const double* znext, const double* znow,
                   const double* f_old, const double* ex_old, const double* ey_old, double* f_new, double* ex_new,
                   double* ey_new, double* z_new, double dt, double m, bool cubic);

// strategy-1 remap of the interval outputs (float64, N x N planes)
void launch_remap_s1(RunView& r, const double* fh, const double* fz, const double* ex, const double* ey,
                     double* out, unsigned* best, int max_extent, unsigned long long* resid_bits);

#define LM_DISPATCH_N_RET(n, out, FN, ...)       \
  switch (n) {                                    \
    case 64: out = FN<64>(__VA_ARGS__); break;    \
    case 128: out = FN<128>(__VA_ARGS__); break;  \
    case 192: out = FN<192>(__VA_ARGS__); break;  \
    case 256: out = FN<256>(__VA_ARGS__); break;  \
    case 384: out = FN<384>(__VA_ARGS__); break;  \
    case 512: out = FN<512>(__VA_ARGS__); break;  \
    case 1024: out = FN<1024>(__VA_ARGS__); break;\
    default: break;                               \
  }

#define LM_DISPATCH_N(n, FN, ...)            \
  switch (n) {                               \
    case 64: FN<64>(__VA_ARGS__); break;     \
    case 128: FN<128>(__VA_ARGS__); break;   \
    case 192: FN<192>(__VA_ARGS__); break;   \
    case 256: FN<256>(__VA_ARGS__); break;   \
    case 384: FN<384>(__VA_ARGS__); break;   \
    case 512: FN<512>(__VA_ARGS__); break;   \
    case 1024: FN<1024>(__VA_ARGS__); break; \
    default: break;                          \
  }

}  // namespace lm
