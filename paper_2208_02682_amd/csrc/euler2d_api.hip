// C ABI of the two-dimensional incompressible flow with strategy 1
// pseudospectral and semi-Lagrangian (lm_e2d_*, include/lagmean.h).  float64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lagmean.h"
#include "launch.hpp"
#include "twiddles.hpp"

using lm::cplx;

namespace lm {
lm_status api_fail(lm_status s, const std::string& msg);
}

namespace {

lm_status fail(lm_status s, const std::string& msg) { return lm::api_fail(s, msg); }

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(LM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

lm_status check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LM_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return LM_OK;
}

constexpr int NS = 11;  // spectral / physical fields of a stage
constexpr int NOUT_E2D = 7;

}  // namespace

struct lm_e2d {
  lm::RunView v;  // dims, stream, slab and twiddles for the transform launchers
  double dt, U0, V0;
  bool cubic;
  // byte offsets in v.slab
  size_t Y, Y1, K1, R, S, IC, PH, NL, RSF, SLf[2], SLx[2], SLy[2], Zn[2], OUT, total;
  int cur;
  bool has_state, in_interval, has_out;
  int64_t n, n_tau;
  double T;
  template <typename X>
  X* at(size_t off) { return reinterpret_cast<X*>(v.slab + off); }
};

namespace {

lm_status e2d_layout(lm_e2d* e) {
  const lm::Dims& d = e->v.d;
  const size_t sp = d.spec_elems(), rf = d.rowfield_elems(), nn = (size_t)d.N * d.N;
  const size_t cD = sizeof(cplx<double>);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t a = o;
    o += (bytes + 255) / 256 * 256;
    return a;
  };
  e->v.L = lm::Layout{};
  e->v.L.tw64 = take(d.N * cD);
  e->Y = take(4 * sp * cD);
  e->Y1 = take(4 * sp * cD);
  e->K1 = take(4 * sp * cD);
  e->R = take(4 * sp * cD);
  e->S = take(NS * sp * cD);
  e->IC = take(NS * rf * cD);
  e->PH = take(NS * nn * sizeof(double));
  e->NL = take(4 * nn * sizeof(double));
  e->RSF = take(4 * rf * cD);
  for (int k = 0; k < 2; ++k) {
    e->SLf[k] = take(nn * sizeof(double));
    e->SLx[k] = take(nn * sizeof(double));
    e->SLy[k] = take(nn * sizeof(double));
    e->Zn[k] = take(nn * sizeof(double));
  }
  e->OUT = take(NOUT_E2D * nn * sizeof(double));
  e->total = o;
  return LM_OK;
}

// spectral inputs -> physical fields: the first `count` of the 11 stage fields
lm_status e2d_to_physical(lm_e2d* e, const cplx<double>* Yin, int count) {
  lm::RunView& v = e->v;
  const lm::Dims& d = v.d;
  const size_t sp = d.spec_elems(), rf = d.rowfield_elems(), nn = (size_t)d.N * d.N;
  cplx<double>* S = e->at<cplx<double>>(e->S);
  cplx<double>* IC = e->at<cplx<double>>(e->IC);
  double* PH = e->at<double>(e->PH);
  lm::launch_e2d_spec(v.stream, d, Yin, S);
  for (int q0 = 0; q0 < count; q0 += lm::IO_MAX) {
    lm::IoColInv J{};
    const int c = std::min(lm::IO_MAX, count - q0);
    for (int q = 0; q < c; ++q) {
      J.src[q] = S + (q0 + q) * sp;
      J.src_f32[q] = 0;
      J.dst[q] = IC + (q0 + q) * rf;
    }
    LM_DISPATCH_N(d.N, lm::launch_io_col_inverse, v, J, c);
  }
  lm::IoRowInv K{};
  int p = 0;
  for (int q = 0; q < count; q += 2, ++p) {
    K.a[p] = IC + q * rf;
    K.oa[p] = PH + q * nn;
    K.sa[p] = 1.0;
    K.ca[p] = (q == 0) ? e->U0 : 0.0;  // u carries the uniform flow
    if (q + 1 < count) {
      K.b[p] = IC + (q + 1) * rf;
      K.ob[p] = PH + (q + 1) * nn;
      K.sb[p] = 1.0;
      K.cb[p] = (q == 0) ? e->V0 : 0.0;
    }
  }
  LM_DISPATCH_N(d.N, lm::launch_io_row_inverse, v, K, p);
  return check_launch();
}

// right-hand sides of the vorticity, g~, P_x, P_y at state Yin and time s since tau
lm_status e2d_rhs(lm_e2d* e, const cplx<double>* Yin, double s) {
  lm::RunView& v = e->v;
  const lm::Dims& d = v.d;
  const size_t sp = d.spec_elems(), rf = d.rowfield_elems(), nn = (size_t)d.N * d.N;
  lm_status st;
  if ((st = e2d_to_physical(e, Yin, NS)) != LM_OK) return st;
  double* NL = e->at<double>(e->NL);
  lm::launch_e2d_products(v.stream, (int)nn, e->at<double>(e->PH), NL, s);
  cplx<double>* RSF = e->at<cplx<double>>(e->RSF);
  lm::IoRowFwd F{};
  for (int p = 0; p < 2; ++p) {
    F.a[p] = NL + (2 * p) * nn;
    F.b[p] = NL + (2 * p + 1) * nn;
    F.oa[p] = RSF + (2 * p) * rf;
    F.ob[p] = RSF + (2 * p + 1) * rf;
  }
  LM_DISPATCH_N(d.N, lm::launch_io_row_forward, v, F, 2);
  lm::IoColFwd C{};
  cplx<double>* R = e->at<cplx<double>>(e->R);
  for (int q = 0; q < 4; ++q) {
    C.src[q] = RSF + q * rf;
    C.dst[q] = R + q * sp;
    C.dst_f32[q] = 0;
  }
  LM_DISPATCH_N(d.N, lm::launch_io_col_forward, v, C, 4);
  return check_launch();
}

lm_status e2d_zero_means(lm_e2d* e) {
  const size_t sp = e->v.d.spec_elems(), nn = (size_t)e->v.d.N * e->v.d.N;
  HIP_TRY(hipMemsetAsync(e->at<char>(e->Y) + sp * sizeof(cplx<double>), 0, 3 * sp * sizeof(cplx<double>), e->v.stream));
  HIP_TRY(hipMemsetAsync(e->at<char>(e->SLf[e->cur]), 0, nn * sizeof(double), e->v.stream));
  HIP_TRY(hipMemsetAsync(e->at<char>(e->SLx[e->cur]), 0, nn * sizeof(double), e->v.stream));
  HIP_TRY(hipMemsetAsync(e->at<char>(e->SLy[e->cur]), 0, nn * sizeof(double), e->v.stream));
  return LM_OK;
}

// one Heun step of everything, then the semi-Lagrangian update; the events
// ev0, ev1 (may be null) bracket the semi-Lagrangian kernel
lm_status e2d_one_step(lm_e2d* e, hipEvent_t ev0, hipEvent_t ev1) {
  lm::RunView& v = e->v;
  const lm::Dims& d = v.d;
  const size_t sp = d.spec_elems(), nn = (size_t)d.N * d.N;
  const double m = double(e->n - e->n_tau);
  const double s0 = m * e->dt;
  cplx<double>* Y = e->at<cplx<double>>(e->Y);
  cplx<double>* Y1 = e->at<cplx<double>>(e->Y1);
  cplx<double>* K1 = e->at<cplx<double>>(e->K1);
  const cplx<double>* R = e->at<cplx<double>>(e->R);
  lm_status st;
  if ((st = e2d_rhs(e, Y, s0)) != LM_OK) return st;
  lm::launch_e2d_stage(v.stream, sp, Y, Y1, K1, R, e->dt, 0);
  if ((st = e2d_rhs(e, Y1, s0 + e->dt)) != LM_OK) return st;
  lm::launch_e2d_stage(v.stream, sp, Y, Y1, K1, R, e->dt, 1);
  // u, v (with the uniform flow) and zeta at t_{n+1}: stage fields 0 .. 4
  if ((st = e2d_to_physical(e, Y, 5)) != LM_OK) return st;
  const double* PH = e->at<double>(e->PH);
  const int c = e->cur, o = c ^ 1;
  if (ev0) HIP_TRY(hipEventRecord(ev0, v.stream));
  lm::launch_e2d_sl(v.stream, d.N, PH, PH + nn, PH + 4 * nn, e->at<double>(e->Zn[c]), e->at<double>(e->SLf[c]),
                    e->at<double>(e->SLx[c]), e->at<double>(e->SLy[c]), e->at<double>(e->SLf[o]),
                    e->at<double>(e->SLx[o]), e->at<double>(e->SLy[o]), e->at<double>(e->Zn[o]), e->dt, m, e->cubic);
  if (ev1) HIP_TRY(hipEventRecord(ev1, v.stream));
  e->cur = o;
  e->n += 1;
  return check_launch();
}

}  // namespace

extern "C" {

lm_status lm_e2d_create(const lm_e2d_config* cfg, void* hip_stream, lm_e2d** out) {
  if (!out) return fail(LM_E_ARG, "null out");
  *out = nullptr;
  if (!cfg) return fail(LM_E_ARG, "null config");
  const int n = cfg->n;
  if (!(n == 64 || n == 128 || n == 192 || n == 256 || n == 384 || n == 512 || n == 1024))
    return fail(LM_E_UNSUPPORTED, "n must be 64, 128, 192, 256, 384, 512 or 1024");
  if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return fail(LM_E_ARG, "dt must be positive and finite");
  if (!std::isfinite(cfg->U0) || !std::isfinite(cfg->V0)) return fail(LM_E_ARG, "U0, V0 must be finite");
  if (cfg->interp != LM_INTERP_BILINEAR && cfg->interp != LM_INTERP_CUBIC)
    return fail(LM_E_UNSUPPORTED, "interp must be LM_INTERP_BILINEAR or LM_INTERP_CUBIC");
  lm_e2d* e = new lm_e2d();
  e->v.d = lm::Dims::make(n);
  e->v.stream = (hipStream_t)hip_stream;
  e->v.fp32 = false;
  e->v.cubic = false;
  e->dt = cfg->dt;
  e->U0 = cfg->U0;
  e->V0 = cfg->V0;
  e->cubic = cfg->interp == LM_INTERP_CUBIC;
  e->cur = 0;
  e->has_state = e->in_interval = e->has_out = false;
  e->n = e->n_tau = 0;
  e->T = 0.0;
  e2d_layout(e);
  hipError_t err = hipMalloc((void**)&e->v.slab, e->total);
  if (err != hipSuccess) {
    delete e;
    (void)hipGetLastError();
    return fail(LM_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(err));
  }
  const std::vector<cplx<double>> tw = lm::stage_twiddles<double>(n);
  err = hipMemcpy(e->v.slab + e->v.L.tw64, tw.data(), n * sizeof(cplx<double>), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(e->v.slab);
    delete e;
    return fail(LM_E_HIP, std::string("twiddles: ") + hipGetErrorString(err));
  }
  *out = e;
  return LM_OK;
}

lm_status lm_e2d_set_vorticity(lm_e2d* e, const double* zeta, int on_device) {
  if (!e || !zeta) return fail(LM_E_ARG, "null argument");
  lm::RunView& v = e->v;
  const lm::Dims& d = v.d;
  const size_t sp = d.spec_elems(), rf = d.rowfield_elems(), nn = (size_t)d.N * d.N;
  const lm::StreamDrain drain{v.stream};  // the caller's buffer is read before any return
  double* PH = e->at<double>(e->PH);
  HIP_TRY(hipMemcpyAsync(PH, zeta, nn * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         v.stream));
  cplx<double>* RSF = e->at<cplx<double>>(e->RSF);
  lm::IoRowFwd F{};
  F.a[0] = PH;
  F.oa[0] = RSF;
  LM_DISPATCH_N(d.N, lm::launch_io_row_forward, v, F, 1);
  lm::IoColFwd C{};
  C.src[0] = RSF;
  C.dst[0] = e->at<cplx<double>>(e->Y);
  C.dst_f32[0] = 0;
  LM_DISPATCH_N(d.N, lm::launch_io_col_forward, v, C, 1);
  e->cur = 0;
  lm_status st;
  if ((st = e2d_zero_means(e)) != LM_OK) return st;
  // zeta_n on the grid for the first semi-Lagrangian step
  if ((st = e2d_to_physical(e, e->at<cplx<double>>(e->Y), 5)) != LM_OK) return st;
  HIP_TRY(hipMemcpyAsync(e->at<double>(e->Zn[e->cur]), PH + 4 * nn, nn * sizeof(double), hipMemcpyDeviceToDevice,
                         v.stream));
  (void)sp;
  HIP_TRY(hipStreamSynchronize(v.stream));
  e->n = e->n_tau = 0;
  e->has_state = true;
  e->in_interval = false;
  return LM_OK;
}

lm_status lm_e2d_begin_interval(lm_e2d* e) {
  if (!e) return fail(LM_E_ARG, "null handle");
  if (!e->has_state) return fail(LM_E_STATE, "no vorticity set");
  lm_status st;
  if ((st = e2d_zero_means(e)) != LM_OK) return st;
  e->n_tau = e->n;
  e->in_interval = true;
  return LM_OK;
}

lm_status lm_e2d_step(lm_e2d* e, int32_t nsteps) {
  if (!e) return fail(LM_E_ARG, "null handle");
  if (nsteps < 0) return fail(LM_E_ARG, "nsteps < 0");
  if (!e->has_state) return fail(LM_E_STATE, "no vorticity set");
  for (int k = 0; k < nsteps; ++k) {
    lm_status st = e2d_one_step(e, nullptr, nullptr);
    if (st != LM_OK) return st;
  }
  return LM_OK;
}

lm_status lm_e2d_step_profiled(lm_e2d* e, int32_t nsteps, double* ms_step, double* ms_sl) {
  if (!e || !ms_step || !ms_sl) return fail(LM_E_ARG, "null argument");
  if (nsteps <= 0 || nsteps > 4096) return fail(LM_E_ARG, "nsteps must be in 1..4096");
  if (!e->has_state) return fail(LM_E_STATE, "no vorticity set");
  std::vector<hipEvent_t> ev(2 * nsteps + 2, nullptr);
  lm_status st = LM_OK;
  for (auto& x : ev)
    if (hipEventCreateWithFlags(&x, hipEventDisableSystemFence) != hipSuccess) st = fail(LM_E_HIP, "event creation");
  if (st == LM_OK && hipEventRecord(ev[2 * nsteps], e->v.stream) != hipSuccess) st = fail(LM_E_HIP, "event record");
  for (int k = 0; k < nsteps && st == LM_OK; ++k) st = e2d_one_step(e, ev[2 * k], ev[2 * k + 1]);
  if (st == LM_OK && hipEventRecord(ev[2 * nsteps + 1], e->v.stream) != hipSuccess) st = fail(LM_E_HIP, "event record");
  if (st == LM_OK && hipEventSynchronize(ev[2 * nsteps + 1]) != hipSuccess) st = fail(LM_E_HIP, "event sync");
  if (st == LM_OK) {
    double sl = 0.0;
    float t = 0.f;
    for (int k = 0; k < nsteps; ++k) {
      if (hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]) != hipSuccess) st = fail(LM_E_HIP, "elapsed time");
      sl += t;
    }
    if (hipEventElapsedTime(&t, ev[2 * nsteps], ev[2 * nsteps + 1]) != hipSuccess) st = fail(LM_E_HIP, "elapsed time");
    *ms_step = double(t) / nsteps;
    *ms_sl = sl / nsteps;
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  return st;
}

lm_status lm_e2d_end_interval(lm_e2d* e, double* T_out) {
  if (!e) return fail(LM_E_ARG, "null handle");
  if (!e->in_interval) return fail(LM_E_STATE, "no open interval");
  if (e->n == e->n_tau) return fail(LM_E_STATE, "interval holds no step");
  lm::RunView& v = e->v;
  const lm::Dims& d = v.d;
  const size_t sp = d.spec_elems(), rf = d.rowfield_elems(), nn = (size_t)d.N * d.N;
  const double T = double(e->n - e->n_tau) * e->dt;
  const lm::StreamDrain drain{v.stream};
  cplx<double>* IC = e->at<cplx<double>>(e->IC);
  double* OUT = e->at<double>(e->OUT);
  lm::IoColInv J{};
  for (int q = 0; q < 4; ++q) {
    J.src[q] = e->at<cplx<double>>(e->Y) + q * sp;
    J.src_f32[q] = 0;
    J.dst[q] = IC + q * rf;
  }
  LM_DISPATCH_N(d.N, lm::launch_io_col_inverse, v, J, 4);
  lm::IoRowInv K{};
  for (int p = 0; p < 2; ++p) {
    K.a[p] = IC + (2 * p) * rf;
    K.b[p] = IC + (2 * p + 1) * rf;
    K.oa[p] = OUT + (2 * p) * nn;
    K.ob[p] = OUT + (2 * p + 1) * nn;
    K.sa[p] = (p == 0) ? 1.0 : 1.0 / T;  // zeta itself, then g~ / T; P_x / T, P_y / T
    K.sb[p] = 1.0 / T;
  }
  LM_DISPATCH_N(d.N, lm::launch_io_row_inverse, v, K, 2);
  const size_t plane = nn * sizeof(double);
  HIP_TRY(hipMemcpyAsync(OUT + 4 * nn, e->at<double>(e->SLf[e->cur]), plane, hipMemcpyDeviceToDevice, v.stream));
  HIP_TRY(hipMemcpyAsync(OUT + 5 * nn, e->at<double>(e->SLx[e->cur]), plane, hipMemcpyDeviceToDevice, v.stream));
  HIP_TRY(hipMemcpyAsync(OUT + 6 * nn, e->at<double>(e->SLy[e->cur]), plane, hipMemcpyDeviceToDevice, v.stream));
  lm_status st;
  if ((st = check_launch()) != LM_OK) return st;
  HIP_TRY(hipStreamSynchronize(v.stream));
  e->T = T;
  e->has_out = true;
  e->in_interval = false;
  if (T_out) *T_out = T;
  return LM_OK;
}

lm_status lm_e2d_read(lm_e2d* e, int32_t kind, double* out, int on_device) {
  if (!e || !out) return fail(LM_E_ARG, "null argument");
  if (kind < LM_E2D_ZETA || kind > LM_E2D_SL_ETA_Y) return fail(LM_E_ARG, "unknown kind");
  if (!e->has_out) return fail(LM_E_STATE, "no closed interval");
  const lm::StreamDrain drain{e->v.stream};  // the caller's buffer is written before any return
  const size_t nn = (size_t)e->v.d.N * e->v.d.N;
  HIP_TRY(hipMemcpyAsync(out, e->at<double>(e->OUT) + kind * nn, nn * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, e->v.stream));
  HIP_TRY(hipStreamSynchronize(e->v.stream));
  return LM_OK;
}

lm_status lm_e2d_destroy(lm_e2d* e) {
  if (!e) return LM_OK;
  hipError_t err = hipStreamSynchronize(e->v.stream);
  (void)hipFree(e->v.slab);
  delete e;
  if (err != hipSuccess) return fail(LM_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(err));
  return LM_OK;
}

}  // extern "C"
