// Definitions of the per-N launchers declared in launch.hpp.
#pragma once

#include <type_traits>
#include <vector>

#include "io_kernels.hpp"
#include "launch.hpp"
#include "step_kernels.hpp"

namespace lm {

// does nothing; used to separate timed launches
template <int N>
__global__ void k_drain() {}

template <int N>
dim3 row_grid(int tasks) {
  return dim3(N / RowGeo<N>::RPB, tasks);
}
// the dynamics rows pass (its block shape depends on the precision)
template <typename T, int N>
dim3 dyn_grid() {
  return dim3(N / DynGeo<T, N>::RPB);
}
template <typename T, int N>
dim3 dyn_block() {
  return dim3(DynGeo<T, N>::THREADS);
}
template <int N, int W = 0>
dim3 col_grid(const Dims& d, int groups) {
  constexpr int C = col_tile<N, W>();
  return dim3((d.NKX + C - 1) / C, groups);
}
template <int N, int W = 0>
dim3 col_block() {
  return dim3(col_threads<N, W>());
}

// calls go(std::integral_constant<int, W>) with the schedule's tile width W
// (the default width if that one is not usable for this N and precision)
template <typename T, int N, typename F>
void with_tile(int tile, F&& go) {
  constexpr int cb = (int)sizeof(cplx<T>);
  if constexpr (col_tile_usable(N, -1, cb)) {
    if (tile < 0) return go(std::integral_constant<int, -1>{});
  }
  if constexpr (col_tile_usable(N, 1, cb)) {
    if (tile > 0) return go(std::integral_constant<int, 1>{});
  }
  go(std::integral_constant<int, 0>{});
}

// the column groups in slots [first, first + count) of one stage, on stream st
// (the stage-value buffers are flipped by the caller once per stage)
template <typename T, int N>
void launch_columns_part(RunView& r, int stage, int first, int count, hipStream_t st) {
  const StepPtrs<T> P = step_ptrs<T>(r);
  cplx<T>* Ys[2] = {(cplx<T>*)r.at(r.L.Ys0), (cplx<T>*)r.at(r.L.Ys1)};
  const cplx<T>* Ys_in = Ys[r.ys_cur];
  cplx<T>* Ys_out = (stage < 0) ? Ys[r.ys_cur] : Ys[r.ys_cur ^ 1];
  // time of the stage input this launch prepares: the current one in the
  // prologue, else the next stage's (c = 1/2, 1/2, 1, then the next step's 0)
  const double t_next = (double(r.n) + (stage < 0 ? 0.0 : (stage <= 1 ? 0.5 : 1.0))) * r.ph.dt;
  with_tile<T, N>(r.sched.tile, [&](auto w) {
    constexpr int W = decltype(w)::value;
    const dim3 g = col_grid<N, W>(r.d, count), b = col_block<N, W>();
    hipLaunchKernelGGL((k_columns<T, N, W>), g, b, 0, st, P, r.d, r.ph, stage, t_next, Ys_in, Ys_out,
                       r.sched.remap, first);
  });
}

template <typename T, int N>
void launch_columns_t(RunView& r, int stage) {
  launch_columns_part<T, N>(r, stage, 0, col_groups(r.ph), r.stream);
  if (stage >= 0) r.ys_cur ^= 1;
}

// the rows pass of the mean right-hand sides, and the momentum rows when requested
template <typename T, int N>
void launch_rows_rhs(RunView& r, const StepPtrs<T>& P, double sval) {
  const dim3 g = row_grid<N>(rhs_tasks<T, N>()), b(64 * ROW_WAVES);
  const int rm = r.sched.remap;
  const int src = r.ph.gen;  // strategy-1 sources in the rows pass only for other averaged fields
  if (r.cubic) hipLaunchKernelGGL((k_rows_rhs<T, N, true>), g, b, 0, r.stream, P, r.d, sval, rm, src);
  else hipLaunchKernelGGL((k_rows_rhs<T, N, false>), g, b, 0, r.stream, P, r.d, sval, rm, src);
  if (r.mom) {
    const dim3 gm = row_grid<N>(2);
    if (r.cubic) hipLaunchKernelGGL((k_rows_mom<T, N, true>), gm, b, 0, r.stream, P, r.d, sval, rm);
    else hipLaunchKernelGGL((k_rows_mom<T, N, false>), gm, b, 0, r.stream, P, r.d, sval, rm);
  }
}

// Two-stream form of the steps.  Per stage the dependencies are
//   rows_dyn(i)  <- the dynamics column groups of stage i-1 (their outputs),
//                   rows_rhs(i-1) (it reads the physical fields rows_dyn rewrites)
//                   and the mean column groups of stage i-1 (the strategy-1
//                   sources and Eulerian accumulators among them read the stage
//                   values that the dynamics groups of stage i overwrite),
//   rows_rhs(i)  <- rows_dyn(i) and the mean column groups of stage i-1,
//   dynamics column groups(i) <- rows_dyn(i),  mean column groups(i) <- rows_rhs(i),
// and no pass writes what a pass it may overlap with reads.  The auxiliary
// stream carries rows_dyn and the dynamics groups, the run's stream rows_rhs
// and the mean groups, so the dynamics groups overlap rows_rhs and the mean
// groups.  Same kernels, same arguments, same results as the one-stream form.
template <typename T, int N>
hipError_t launch_steps_2s(RunView& r, int nsteps) {
  const StepPtrs<T> P = step_ptrs<T>(r);
  static const double c[4] = {0.0, 0.5, 0.5, 1.0};
  const int nd = col_dyn_groups(r.ph), nm = col_mean_groups(r.ph);
  hipEvent_t fork = r.ev[0], dyn = r.ev[1], rhs = r.ev[2], join = r.ev[3];
  hipError_t e = hipEventRecord(fork, r.stream);  // aux starts after everything queued so far
  if (e == hipSuccess) e = hipStreamWaitEvent(r.aux, fork, 0);
  for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
    for (int stage = 0; stage < 4 && e == hipSuccess; ++stage) {
      const double sval = (double(r.n - r.n_tau) + c[stage]) * r.ph.dt;
      // the previous stage's run-stream work: rows_rhs reads the physical
      // fields rows_dyn rewrites, and the mean groups read the stage values the
      // next dynamics groups overwrite
      if (s + stage > 0) e = hipStreamWaitEvent(r.aux, rhs, 0);
      if (e != hipSuccess) break;
      hipLaunchKernelGGL((k_rows_dyn<T, N>), (dyn_grid<T, N>()), (dyn_block<T, N>()), 0, r.aux, P, r.d, r.ph,
                         r.sched.remap);
      e = hipEventRecord(dyn, r.aux);
      launch_columns_part<T, N>(r, stage, 0, nd, r.aux);
      if (e == hipSuccess) e = hipStreamWaitEvent(r.stream, dyn, 0);
      if (e != hipSuccess) break;
      launch_rows_rhs<T, N>(r, P, sval);  // on the run's stream
      launch_columns_part<T, N>(r, stage, nd, nm, r.stream);
      e = hipEventRecord(rhs, r.stream);
      r.ys_cur ^= 1;
    }
    r.n += 1;
  }
  // the run's stream resumes after the auxiliary stream's last work
  const hipError_t e2 = hipEventRecord(join, r.aux);
  const hipError_t e3 = (e2 == hipSuccess) ? hipStreamWaitEvent(r.stream, join, 0) : e2;
  return e != hipSuccess ? e : e3;
}

template <typename T, int N>
void launch_steps_t(RunView& r, int nsteps) {
  const StepPtrs<T> P = step_ptrs<T>(r);
  static const double c[4] = {0.0, 0.5, 0.5, 1.0};
  if (r.sched.streams == 2 && r.aux && nsteps > 0) {
    (void)launch_steps_2s<T, N>(r, nsteps);  // launch errors surface through hipGetLastError
    return;
  }
  for (int s = 0; s < nsteps; ++s) {
    for (int stage = 0; stage < 4; ++stage) {
      // time since the interval start, from integers
      const double sval = (double(r.n - r.n_tau) + c[stage]) * r.ph.dt;
      hipLaunchKernelGGL((k_rows_dyn<T, N>), (dyn_grid<T, N>()), (dyn_block<T, N>()), 0, r.stream, P, r.d,
                         r.ph, r.sched.remap);
      launch_rows_rhs<T, N>(r, P, sval);
      launch_columns_t<T, N>(r, stage);
    }
    r.n += 1;
  }
}

// Same launches as launch_steps_t, each bracketed by a pair of events on the
// run's stream; nothing synchronises until all steps are enqueued, so the
// kernels run back to back as in launch_steps_t.  The three kernel durations
// are accumulated into ms[0..2].
template <typename T, int N>
hipError_t launch_steps_profiled_t(RunView& r, int nsteps, double* ms) {
  const StepPtrs<T> P = step_ptrs<T>(r);
  static const double c[4] = {0.0, 0.5, 0.5, 1.0};
  const int nev = nsteps * 4 * 3 * 2;
  std::vector<hipEvent_t> ev(nev);
  hipError_t err = hipSuccess;
  int made = 0;
  // device-scope markers: no system-scope cache release around every launch
  for (; made < nev && err == hipSuccess; ++made) err = hipEventCreateWithFlags(&ev[made], hipEventDisableSystemFence);
  if (err != hipSuccess) {
    for (int i = 0; i < made - 1; ++i) (void)hipEventDestroy(ev[i]);
    return err;
  }
  int e = 0;
  for (int s = 0; s < nsteps; ++s) {
    for (int stage = 0; stage < 4; ++stage) {
      const double sval = (double(r.n - r.n_tau) + c[stage]) * r.ph.dt;
      // an empty kernel between one kernel's end marker and the next one's
      // start marker absorbs the work done at kernel boundaries, so each
      // interval covers one kernel's execution only
      (void)hipEventRecord(ev[e++], r.stream);
      hipLaunchKernelGGL((k_rows_dyn<T, N>), (dyn_grid<T, N>()), (dyn_block<T, N>()), 0, r.stream, P, r.d,
                         r.ph, r.sched.remap);
      (void)hipEventRecord(ev[e++], r.stream);
      hipLaunchKernelGGL(k_drain<N>, dim3(1), dim3(64), 0, r.stream);
      (void)hipEventRecord(ev[e++], r.stream);
      launch_rows_rhs<T, N>(r, P, sval);
      (void)hipEventRecord(ev[e++], r.stream);
      hipLaunchKernelGGL(k_drain<N>, dim3(1), dim3(64), 0, r.stream);
      (void)hipEventRecord(ev[e++], r.stream);
      launch_columns_t<T, N>(r, stage);
      (void)hipEventRecord(ev[e++], r.stream);
      hipLaunchKernelGGL(k_drain<N>, dim3(1), dim3(64), 0, r.stream);
    }
    r.n += 1;
  }
  err = hipEventSynchronize(ev[nev - 1]);
  for (int i = 0; i < nev && err == hipSuccess; i += 2) {
    float t = 0.f;
    err = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
    ms[(i / 2) % 3] += t;
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  return err;
}

template <int N>
hipError_t launch_steps_profiled(RunView& r, int nsteps, double* ms) {
  if (r.fp32) return launch_steps_profiled_t<float, N>(r, nsteps, ms);
  return launch_steps_profiled_t<double, N>(r, nsteps, ms);
}

// one RK4 step of every run of one (N, precision) group: blockIdx.z selects
// the run's descriptor
template <typename T, int N>
void launch_batch_step_t(hipStream_t st, const RunDesc<T>* desc, int nruns, bool cubic, bool mom, int ncg,
                         const Sched& sc) {
  const Dims d = Dims::make(N);
  const int rm = sc.remap;
  for (int stage = 0; stage < 4; ++stage) {
    dim3 g1 = dyn_grid<T, N>();
    g1.z = nruns;
    hipLaunchKernelGGL((k_rows_dyn_b<T, N>), g1, (dyn_block<T, N>()), 0, st, desc, rm);
    dim3 g2 = row_grid<N>(rhs_tasks<T, N>());
    g2.z = nruns;
    const dim3 b2(64 * ROW_WAVES);
    if (cubic) hipLaunchKernelGGL((k_rows_rhs_b<T, N, true>), g2, b2, 0, st, desc, stage, rm);
    else hipLaunchKernelGGL((k_rows_rhs_b<T, N, false>), g2, b2, 0, st, desc, stage, rm);
    if (mom) {
      dim3 gm = row_grid<N>(2);
      gm.z = nruns;
      if (cubic) hipLaunchKernelGGL((k_rows_mom_b<T, N, true>), gm, b2, 0, st, desc, stage, rm);
      else hipLaunchKernelGGL((k_rows_mom_b<T, N, false>), gm, b2, 0, st, desc, stage, rm);
    }
    with_tile<T, N>(sc.tile, [&](auto w) {
      constexpr int W = decltype(w)::value;
      dim3 g3 = col_grid<N, W>(d, ncg);
      g3.z = nruns;
      const dim3 b3 = col_block<N, W>();
      hipLaunchKernelGGL((k_columns_b<T, N, W>), g3, b3, 0, st, desc, stage, rm);
    });
  }
}

template <int N>
void launch_batch_step(hipStream_t st, const void* desc, int nruns, bool fp32, bool cubic, bool mom, int ncg,
                       const Sched& sc) {
  if (fp32) launch_batch_step_t<float, N>(st, (const RunDesc<float>*)desc, nruns, cubic, mom, ncg, sc);
  else launch_batch_step_t<double, N>(st, (const RunDesc<double>*)desc, nruns, cubic, mom, ncg, sc);
}

template <int N>
void launch_steps(RunView& r, int nsteps) {
  if (r.fp32) launch_steps_t<float, N>(r, nsteps);
  else launch_steps_t<double, N>(r, nsteps);
}

template <int N>
void launch_prologue(RunView& r) {
  if (r.fp32) launch_columns_t<float, N>(r, -1);
  else launch_columns_t<double, N>(r, -1);
}

template <int N>
void launch_io_col_inverse(RunView& r, const IoColInv& J, int count) {
  hipLaunchKernelGGL((k_io_col_inverse<N>), col_grid<N>(r.d, count), col_block<N>(), 0, r.stream, J, r.d,
                     (const cplx<double>*)r.at(r.L.tw64));
}
template <int N>
void launch_io_row_inverse(RunView& r, const IoRowInv& J, int count) {
  hipLaunchKernelGGL((k_io_row_inverse<N>), row_grid<N>(count), dim3(64 * ROW_WAVES), 0, r.stream, J, r.d,
                     (const cplx<double>*)r.at(r.L.tw64));
}
template <int N>
void launch_io_row_forward(RunView& r, const IoRowFwd& J, int count) {
  hipLaunchKernelGGL((k_io_row_forward<N>), row_grid<N>(count), dim3(64 * ROW_WAVES), 0, r.stream, J, r.d,
                     (const cplx<double>*)r.at(r.L.tw64));
}
template <int N>
void launch_io_col_forward(RunView& r, const IoColFwd& J, int count) {
  hipLaunchKernelGGL((k_io_col_forward<N>), col_grid<N>(r.d, count), col_block<N>(), 0, r.stream, J, r.d,
                     (const cplx<double>*)r.at(r.L.tw64));
}

}  // namespace lm

// The per-precision step launchers (and with them every time-stepping kernel)
// are instantiated in inst_<N>_f32.hip and inst_<N>_f64.hip, the dispatchers
// and the float64 boundary launchers in inst_<N>.hip: three translation units
// per grid size compile in parallel.
#define LM_INSTANTIATE_T(T, N)                                                                           \
  namespace lm {                                                                                         \
  template void launch_steps_t<T, N>(RunView&, int);                                                     \
  template hipError_t launch_steps_profiled_t<T, N>(RunView&, int, double*);                             \
  template void launch_columns_t<T, N>(RunView&, int);                                                   \
  template void launch_batch_step_t<T, N>(hipStream_t, const RunDesc<T>*, int, bool, bool, int, const Sched&); \
  }

#define LM_EXTERN_T(T, N)                                                                                       \
  namespace lm {                                                                                                \
  extern template void launch_steps_t<T, N>(RunView&, int);                                                     \
  extern template hipError_t launch_steps_profiled_t<T, N>(RunView&, int, double*);                             \
  extern template void launch_columns_t<T, N>(RunView&, int);                                                   \
  extern template void launch_batch_step_t<T, N>(hipStream_t, const RunDesc<T>*, int, bool, bool, int, const Sched&); \
  }

#define LM_INSTANTIATE(N)                                                                             \
  LM_EXTERN_T(float, N)                                                                               \
  LM_EXTERN_T(double, N)                                                                              \
  namespace lm {                                                                                      \
  template void launch_steps<N>(RunView&, int);                                                       \
  template void launch_batch_step<N>(hipStream_t, const void*, int, bool, bool, bool, int, const Sched&); \
  template hipError_t launch_steps_profiled<N>(RunView&, int, double*);                               \
  template void launch_prologue<N>(RunView&);                                                         \
  template void launch_io_row_forward<N>(RunView&, const IoRowFwd&, int);                             \
  template void launch_io_col_forward<N>(RunView&, const IoColFwd&, int);                             \
  template void launch_io_col_inverse<N>(RunView&, const IoColInv&, int);                             \
  template void launch_io_row_inverse<N>(RunView&, const IoRowInv&, int);                             \
  }
