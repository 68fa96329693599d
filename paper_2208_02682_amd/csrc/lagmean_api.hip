// C ABI of the Lagrangian-mean library: argument checking, run management and
// the order of launches.  The kernels are launched through the per-N launchers
// (launch.hpp); hot-path kernels are in step_kernels.hpp, boundary transforms in
// io_kernels.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <utility>
#include <algorithm>
#include <mutex>
#include <vector>

#include "lagmean.h"
#include "launch.hpp"
#include "twiddles.hpp"

using lm::cplx;

namespace {

thread_local std::string g_err;

lm_status fail(lm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(LM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool supported_n(int n) {
  return n == 64 || n == 128 || n == 192 || n == 256 || n == 384 || n == 512 || n == 1024;
}

lm_status check_cfg(const lm_config* cfg) {
  if (!cfg) return fail(LM_E_ARG, "null config");
  if (!supported_n(cfg->n)) return fail(LM_E_UNSUPPORTED, "n must be 64, 128, 192, 256, 384, 512 or 1024");
  if (cfg->precision != LM_FP64 && cfg->precision != LM_FP32_MIXED)
    return fail(LM_E_ARG, "precision must be LM_FP64 or LM_FP32_MIXED");
  if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return fail(LM_E_ARG, "dt must be positive and finite");
  if (!(cfg->nu8 >= 0.0) || !std::isfinite(cfg->nu8)) return fail(LM_E_ARG, "nu8 must be >= 0");
  if (!std::isfinite(cfg->f) || !std::isfinite(cfg->g) || !std::isfinite(cfg->H))
    return fail(LM_E_ARG, "f, g, H must be finite");
  {
    const uint32_t f = cfg->avg_fields & ~LM_F_MOMENTUM;
    const uint32_t known = LM_F_H | LM_F_ZETA | LM_F_U | LM_F_V | LM_F_Q;
    if ((f & ~known) != 0 || (f != 0 && __builtin_popcount(f) != 2))
      return fail(LM_E_UNSUPPORTED, "averaged fields: two of LM_F_H, LM_F_ZETA, LM_F_U, LM_F_V, LM_F_Q (or 0), "
                                    "optionally with LM_F_MOMENTUM");
  }
  if (cfg->strategies != 0 && cfg->strategies != (LM_S1 | LM_S2 | LM_EULER))
    return fail(LM_E_UNSUPPORTED, "all of strategy 1, strategy 2 and the Eulerian mean are integrated");
  if (cfg->interp != LM_INTERP_BILINEAR && cfg->interp != LM_INTERP_CUBIC)
    return fail(LM_E_UNSUPPORTED, "interp must be LM_INTERP_BILINEAR or LM_INTERP_CUBIC");
  if (cfg->mode != LM_DYNAMIC && cfg->mode != LM_KINEMATIC_PLANEWAVE)
    return fail(LM_E_UNSUPPORTED, "mode must be LM_DYNAMIC or LM_KINEMATIC_PLANEWAVE");
  if (cfg->mode == LM_KINEMATIC_PLANEWAVE) {
    for (int i = 0; i < 7; ++i)
      if (!std::isfinite(cfg->kin[i])) return fail(LM_E_ARG, "kin[] must be finite");
    const double kx = cfg->kin[0], ky = cfg->kin[1];
    const int K = (cfg->n - 1) / 3;
    if (kx != std::floor(kx) || ky != std::floor(ky) || std::fabs(kx) > K || std::fabs(ky) > K)
      return fail(LM_E_ARG, "kin: the wave vector must be integer and inside the 2/3-rule mask");
    if (!(cfg->H > 0.0)) return fail(LM_E_ARG, "kin: H must be positive");
    if (cfg->kin[2] != 0.0 && kx == 0.0 && ky == 0.0) return fail(LM_E_ARG, "kin: a wave needs a wave vector");
  }
  return LM_OK;
}

// the two averaged fields (lowest mask bit first) as lm::FieldSel
void field_slots(uint32_t mask, int* fs0, int* fs1) {
  uint32_t f = mask & ~LM_F_MOMENTUM;
  if (f == 0) f = LM_F_H | LM_F_ZETA;
  static const uint32_t bit[5] = {LM_F_H, LM_F_ZETA, LM_F_U, LM_F_V, LM_F_Q};
  static const int sel[5] = {lm::FS_ETA, lm::FS_ZETA, lm::FS_U, lm::FS_V, lm::FS_Q};
  int k = 0;
  for (int i = 0; i < 5; ++i)
    if (f & bit[i]) (k++ == 0 ? *fs0 : *fs1) = sel[i];
}

// physics constants and launch flags of a valid configuration
lm::Phys make_phys(const lm_config* cfg) {
  lm::Phys ph{};
  ph.f = cfg->f;
  ph.g = cfg->g;
  ph.H = cfg->H;
  ph.dt = cfg->dt;
  ph.nu8 = cfg->nu8;
  field_slots(cfg->avg_fields, &ph.fs0, &ph.fs1);
  ph.gen = !(ph.fs0 == lm::FS_ETA && ph.fs1 == lm::FS_ZETA);
  ph.mom = (cfg->avg_fields & LM_F_MOMENTUM) != 0;
  ph.kin = cfg->mode == LM_KINEMATIC_PLANEWAVE;
  if (ph.kin) {
    ph.kx = cfg->kin[0];
    ph.ky = cfg->kin[1];
    ph.A = cfg->kin[2];
    // omega = 0 asks for the Poincare dispersion relation
    ph.omega = cfg->kin[3] != 0.0 ? cfg->kin[3]
                                  : std::sqrt(cfg->f * cfg->f + cfg->g * cfg->H * (ph.kx * ph.kx + ph.ky * ph.ky));
    ph.phase = cfg->kin[4];
    ph.U0 = cfg->kin[5];
    ph.V0 = cfg->kin[6];
  }
  return ph;
}

// ---------------------------------------------------------------------------
// launch schedules, one per (grid size, precision); every launch reads them
// ---------------------------------------------------------------------------
std::mutex g_sched_mu;
lm::Sched g_sched[2][7][2];  // [0 single runs, 1 batched launches][size index][fp32]
unsigned g_sched_gen = 0;    // bumped on every change: batches re-capture their graph

int size_index(int n) {
  switch (n) {
    case 64: return 0;
    case 128: return 1;
    case 192: return 2;
    case 256: return 3;
    case 384: return 4;
    case 512: return 5;
    case 1024: return 6;
  }
  return -1;
}

lm::Sched get_sched(int n, bool fp32, bool batched, unsigned* gen = nullptr) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  if (gen) *gen = g_sched_gen;
  return g_sched[batched ? 1 : 0][size_index(n)][fp32 ? 1 : 0];
}

void put_sched(int n, bool fp32, bool batched, const lm::Sched& sc) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  g_sched[batched ? 1 : 0][size_index(n)][fp32 ? 1 : 0] = sc;
  ++g_sched_gen;
}

unsigned sched_gen() {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  return g_sched_gen;
}

// the usable schedules of (n, precision), the default first
// (a batch replays captured graphs on its own streams: one-stream schedules only)
std::vector<lm::Sched> sched_candidates(int n, bool fp32, bool batched = false) {
  std::vector<lm::Sched> out;
  const int cb = fp32 ? (int)sizeof(cplx<float>) : (int)sizeof(cplx<double>);
  for (int streams : {1, 2}) {
    if (batched && streams != 1) continue;
    for (int tile : {0, -1, 1}) {
      if (!lm::col_tile_usable(n, tile, cb)) continue;
      for (int remap : {1, 0}) {
        lm::Sched sc;
        sc.tile = tile;
        sc.remap = remap;
        sc.streams = streams;
        out.push_back(sc);
      }
    }
  }
  return out;
}

}  // namespace

struct lm_run : lm::RunView {
  lm_config cfg;
  bool has_state, in_interval, has_mean, has_remap;
  double T;
  lm_batch* batch;  // the batch this run belongs to, if any
};

struct lm_batch {
  struct Member {
    lm_run* run;
    int32_t remaining;
  };
  struct Group {
    int N;
    bool fp32;
    bool cubic;
    bool mom;
    bool gen;  // Eulerian means of fields other than (h, zeta): two more column groups
    void* d_desc = nullptr;  // device array of RunDesc<T>
    size_t cap = 0;          // bytes
    hipStream_t fork = nullptr;
    hipEvent_t join = nullptr;
  };
  hipStream_t user;     // the caller's stream (ordering only)
  hipStream_t stream;   // the batch's own stream: graphs are captured and launched here
  std::vector<Member> members;
  std::vector<Group> groups;
  long long* d_counters = nullptr;  // one per member slot
  int counter_cap = 0;
  hipEvent_t fork_ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<lm_run*> signature;  // active members the graph was built for
  unsigned sched_gen = 0;          // schedule table generation the graph was captured with
  // host image of the device scratch of lm_batch_step_static (descriptors and
  // counters are copied from here; it lives as long as the batch, so the copies
  // never read freed host memory)
  alignas(256) unsigned char static_stage[128 * 1024];
};

namespace {

// the launches of a run follow the table's schedule of its (N, precision)
void use_sched(lm_run* r) { r->sched = get_sched(r->d.N, r->fp32, false); }

// the two-stream schedule's stream (after its work) and events
void release_streams(lm_run* r) {
  if (r->aux) {
    (void)hipStreamSynchronize(r->aux);
    (void)hipStreamDestroy(r->aux);
    r->aux = nullptr;
  }
  for (auto& ev : r->ev) {
    if (ev) (void)hipEventDestroy(ev);
    ev = nullptr;
  }
}

// one prognostic field's storage: leading words, trailing words of a
// compensated float field (else null), and whether it is float
struct FieldRef {
  const void* ptr;
  const void* lo;
  int f32;
};

// working-precision state field sf (lm::StateField)
FieldRef real_field(lm_run* r, int sf) {
  const size_t sp = r->d.spec_elems();
  const size_t cT = r->fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  return {r->slab + r->L.Yr + sf * sp * cT, r->fp32 ? r->slab + r->L.Yl + sf * sp * cT : nullptr,
          r->fp32 ? 1 : 0};
}

FieldRef state_field(lm_run* r, int which) {
  static const int rmap[9] = {lm::SF_U, lm::SF_V, lm::SF_H, lm::SF_GBH, lm::SF_GBZ,
                              lm::SF_GTH, lm::SF_GTZ, lm::SF_EH, lm::SF_EZ};
  if (r->ph.kin && which >= LM_P_U && which <= LM_P_H) {
    // a prescribed flow has no u, v, h state: its values at the current time
    // are the current stage input
    const size_t sp = r->d.spec_elems();
    const size_t cT = r->fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
    const size_t ys = r->ys_cur ? r->L.Ys1 : r->L.Ys0;
    return {r->slab + ys + (which - LM_P_U) * sp * cT, nullptr, r->fp32 ? 1 : 0};
  }
  if (which >= LM_P_U && which <= LM_P_E_ZETA) return real_field(r, rmap[which]);
  const size_t sp = r->d.spec_elems();
  static const int dmap[4] = {lm::SD_XIX, lm::SD_XIY, lm::SD_PX, lm::SD_PY};
  return {r->slab + r->L.Yd + dmap[which - LM_P_XI_X] * sp * sizeof(cplx<double>), nullptr, 0};
}

lm_status copy_in(lm_run* r, double* dst, const double* src, int on_device) {
  const size_t bytes = (size_t)r->d.N * r->d.N * sizeof(double);
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, r->stream));
  return LM_OK;
}
lm_status copy_out(lm_run* r, double* dst, const double* src, int on_device) {
  const size_t bytes = (size_t)r->d.N * r->d.N * sizeof(double);
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, r->stream));
  return LM_OK;
}

lm_status zero_means(lm_run* r) {
  const size_t sp = r->d.spec_elems();
  const size_t cT = r->fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  const int nsf = r->mom ? lm::NSF_R : lm::SF_GMX;
  HIP_TRY(hipMemsetAsync(r->slab + r->L.Yr + lm::SF_GBH * sp * cT, 0, (nsf - lm::SF_GBH) * sp * cT, r->stream));
  if (r->fp32)
    HIP_TRY(hipMemsetAsync(r->slab + r->L.Yl + lm::SF_GBH * sp * cT, 0, (nsf - lm::SF_GBH) * sp * cT, r->stream));
  HIP_TRY(hipMemsetAsync(r->slab + r->L.Yd, 0, lm::NSF_D * sp * sizeof(cplx<double>), r->stream));
  return LM_OK;
}

using lm::StreamDrain;

lm_status check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LM_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return LM_OK;
}

}  // namespace

namespace lm {
// the thread-local error of lm_last_error, for the other API source files
__attribute__((visibility("hidden"))) lm_status api_fail(lm_status s, const std::string& msg) { return fail(s, msg); }
}  // namespace lm

extern "C" {

const char* lm_status_str(lm_status s) {
  switch (s) {
    case LM_OK: return "ok";
    case LM_E_ARG: return "invalid argument";
    case LM_E_STATE: return "call out of order";
    case LM_E_OOM: return "out of device memory";
    case LM_E_HIP: return "HIP runtime error";
    case LM_E_NONFINITE: return "non-finite values in the outputs";
    case LM_E_UNSUPPORTED: return "unsupported configuration";
    case LM_E_BUDGET: return "footprint exceeds the budget";
  }
  return "unknown status";
}

const char* lm_last_error(void) { return g_err.c_str(); }

lm_status lm_device_alloc(size_t bytes, void** ptr) {
  if (!ptr) return fail(LM_E_ARG, "null ptr");
  *ptr = nullptr;
  if (bytes == 0) return LM_OK;
  const hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(LM_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return LM_OK;
}

lm_status lm_device_free(void* ptr) {
  if (!ptr) return LM_OK;
  HIP_TRY(hipFree(ptr));
  return LM_OK;
}

lm_status lm_memcpy(void* dst, const void* src, size_t bytes, int32_t kind) {
  if ((!dst || !src) && bytes) return fail(LM_E_ARG, "null pointer");
  hipMemcpyKind k;
  switch (kind) {
    case LM_COPY_HOST_TO_DEVICE: k = hipMemcpyHostToDevice; break;
    case LM_COPY_DEVICE_TO_HOST: k = hipMemcpyDeviceToHost; break;
    case LM_COPY_DEVICE_TO_DEVICE: k = hipMemcpyDeviceToDevice; break;
    default: return fail(LM_E_ARG, "unknown copy kind");
  }
  if (bytes) HIP_TRY(hipMemcpy(dst, src, bytes, k));
  return LM_OK;
}

lm_status lm_device_synchronize(void) {
  HIP_TRY(hipDeviceSynchronize());
  return LM_OK;
}

lm_status lm_copy_bandwidth(size_t bytes, int32_t reps, double* gbps) {
  if (!gbps || bytes == 0 || reps < 1 || reps > 1000) return fail(LM_E_ARG, "bytes > 0, 1 <= reps <= 1000");
  void *a = nullptr, *b = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&a, bytes);
  if (e == hipSuccess) e = hipMalloc(&b, bytes);
  if (e == hipSuccess) e = hipMemset(a, 0, bytes);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, nullptr);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipDeviceSynchronize();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? LM_E_OOM : LM_E_HIP, std::string("copy bandwidth: ") + hipGetErrorString(e));
  }
  *gbps = 2.0 * double(bytes) * reps / (double(ms) * 1e-3) / 1e9;  // bytes read + bytes written
  return LM_OK;
}

lm_status lm_hip_versions(int32_t* built, int32_t* runtime) {
  if (built) *built = (int32_t)HIP_VERSION;
  if (runtime) {
    int v = 0;
    const hipError_t e = hipRuntimeGetVersion(&v);
    if (e != hipSuccess) return fail(LM_E_HIP, std::string("hipRuntimeGetVersion: ") + hipGetErrorString(e));
    *runtime = (int32_t)v;
  }
  return LM_OK;
}

lm_status lm_query_footprint(const lm_config* cfg, size_t* bytes) {
  lm_status s = check_cfg(cfg);
  if (s != LM_OK) return s;
  if (!bytes) return fail(LM_E_ARG, "null bytes");
  const lm::Phys ph = make_phys(cfg);
  *bytes = lm::make_layout(lm::Dims::make(cfg->n), cfg->precision == LM_FP32_MIXED, ph.mom, ph.gen).total;
  return LM_OK;
}

lm_status lm_create(const lm_config* cfg, void* hip_stream, lm_run** out) {
  lm_status s = check_cfg(cfg);
  if (s != LM_OK) return s;
  if (!out) return fail(LM_E_ARG, "null out");
  *out = nullptr;
  lm_run* r = new lm_run();
  r->cfg = *cfg;
  r->d = lm::Dims::make(cfg->n);
  r->ph = make_phys(cfg);
  r->stream = (hipStream_t)hip_stream;
  r->fp32 = cfg->precision == LM_FP32_MIXED;
  r->cubic = cfg->interp == LM_INTERP_CUBIC;
  r->mom = (cfg->avg_fields & LM_F_MOMENTUM) != 0;
  r->L = lm::make_layout(r->d, r->fp32, r->mom, r->ph.gen);
  r->n = r->n_tau = 0;
  r->has_state = r->in_interval = r->has_mean = r->has_remap = false;
  r->T = 0.0;
  r->ys_cur = 0;
  r->slab = nullptr;
  r->batch = nullptr;
  hipError_t e = hipMalloc((void**)&r->slab, r->L.total);
  if (e != hipSuccess) {
    delete r;
    (void)hipGetLastError();
    return fail(LM_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  // the second stream and the events of the two-stream schedule
  e = hipStreamCreateWithFlags(&r->aux, hipStreamNonBlocking);
  for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&r->ev[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    release_streams(r);
    (void)hipFree(r->slab);
    delete r;
    return fail(LM_E_HIP, std::string("stream creation: ") + hipGetErrorString(e));
  }
  // twiddles exp(-2 pi i m / N) in the transforms' stage-by-stage layout
  const int N = r->d.N;
  const std::vector<cplx<double>> tw = lm::stage_twiddles<double>(N);
  const std::vector<cplx<float>> twf = lm::stage_twiddles<float>(N);
  e = hipMemcpy(r->slab + r->L.tw64, tw.data(), N * sizeof(cplx<double>), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = r->fp32 ? hipMemcpy(r->slab + r->L.twT, twf.data(), N * sizeof(cplx<float>), hipMemcpyHostToDevice)
                : hipMemcpy(r->slab + r->L.twT, tw.data(), N * sizeof(cplx<double>), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(r->slab, 0, r->L.tw64);
  if (e == hipSuccess && r->ph.kin) {
    // a prescribed flow is defined from the start (time 0): its column-pass
    // outputs of the current time, as after lm_set_state
    use_sched(r);
    LM_DISPATCH_N(r->d.N, lm::launch_prologue, *r);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    r->has_state = (e == hipSuccess);
  }
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(r->stream);
    release_streams(r);
    (void)hipFree(r->slab);
    delete r;
    return fail(LM_E_HIP, std::string("init: ") + hipGetErrorString(e));
  }
  *out = r;
  return LM_OK;
}

lm_status lm_set_state(lm_run* r, const double* u, const double* v, const double* h, int on_device) {
  if (!r || !u || !v || !h) return fail(LM_E_ARG, "null argument");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  if (r->ph.kin) return fail(LM_E_STATE, "a kinematic run's flow is prescribed");
  const StreamDrain drain{r->stream};  // the caller's buffers are read before any return
  const size_t nn = (size_t)r->d.N * r->d.N;
  double* phys = (double*)r->at(r->L.phys);
  lm_status s;
  if ((s = copy_in(r, phys, u, on_device)) != LM_OK) return s;
  if ((s = copy_in(r, phys + nn, v, on_device)) != LM_OK) return s;
  if ((s = copy_in(r, phys + 2 * nn, h, on_device)) != LM_OK) return s;
  const size_t rf = r->d.rowfield_elems();
  cplx<double>* ioC = (cplx<double>*)r->at(r->L.ioC);
  lm::IoRowFwd J{};
  J.a[0] = phys; J.b[0] = phys + nn; J.oa[0] = ioC; J.ob[0] = ioC + rf;
  J.a[1] = phys + 2 * nn; J.b[1] = nullptr; J.oa[1] = ioC + 2 * rf; J.ob[1] = nullptr;
  LM_DISPATCH_N(r->d.N, lm::launch_io_row_forward, *r, J, 2);
  lm::IoColFwd K{};
  const size_t sp = r->d.spec_elems();
  const size_t cT = r->fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  for (int q = 0; q < 3; ++q) {
    K.src[q] = ioC + q * rf;
    K.dst[q] = r->slab + r->L.Yr + q * sp * cT;  // SF_U, SF_V, SF_H are 0, 1, 2
    K.dst_lo[q] = r->fp32 ? r->slab + r->L.Yl + q * sp * cT : nullptr;
    K.dst_f32[q] = r->fp32 ? 1 : 0;
  }
  LM_DISPATCH_N(r->d.N, lm::launch_io_col_forward, *r, K, 3);
  if ((s = zero_means(r)) != LM_OK) return s;
  r->ys_cur = 0;
  use_sched(r);
  LM_DISPATCH_N(r->d.N, lm::launch_prologue, *r);
  if ((s = check_launch()) != LM_OK) return s;
  HIP_TRY(hipStreamSynchronize(r->stream));
  r->n = r->n_tau = 0;
  r->has_state = true;
  r->in_interval = false;
  return LM_OK;
}

lm_status lm_get_state(lm_run* r, double* u, double* v, double* h, int on_device) {
  if (!r || !u || !v || !h) return fail(LM_E_ARG, "null argument");
  if (!r->has_state) return fail(LM_E_STATE, "no state set");
  const StreamDrain drain{r->stream};  // the caller's buffers are written before any return
  const size_t nn = (size_t)r->d.N * r->d.N, rf = r->d.rowfield_elems();
  cplx<double>* ioC = (cplx<double>*)r->at(r->L.ioC);
  double* phys = (double*)r->at(r->L.phys);
  lm::IoColInv J{};
  for (int q = 0; q < 3; ++q) {
    const FieldRef f = state_field(r, LM_P_U + q);
    J.src[q] = f.ptr;
    J.src_lo[q] = f.lo;
    J.src_f32[q] = f.f32;
    J.dst[q] = ioC + q * rf;
  }
  LM_DISPATCH_N(r->d.N, lm::launch_io_col_inverse, *r, J, 3);
  lm::IoRowInv K{};
  K.a[0] = ioC; K.b[0] = ioC + rf; K.oa[0] = phys; K.ob[0] = phys + nn; K.sa[0] = K.sb[0] = 1.0;
  K.a[1] = ioC + 2 * rf; K.b[1] = nullptr; K.oa[1] = phys + 2 * nn; K.ob[1] = nullptr; K.sa[1] = 1.0;
  LM_DISPATCH_N(r->d.N, lm::launch_io_row_inverse, *r, K, 2);
  lm_status s;
  if ((s = check_launch()) != LM_OK) return s;
  if ((s = copy_out(r, u, phys, on_device)) != LM_OK) return s;
  if ((s = copy_out(r, v, phys + nn, on_device)) != LM_OK) return s;
  if ((s = copy_out(r, h, phys + 2 * nn, on_device)) != LM_OK) return s;
  HIP_TRY(hipStreamSynchronize(r->stream));
  return LM_OK;
}

lm_status lm_begin_interval(lm_run* r) {
  if (!r) return fail(LM_E_ARG, "null run");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  if (!r->has_state) return fail(LM_E_STATE, "no state set");
  lm_status s;
  if ((s = zero_means(r)) != LM_OK) return s;
  use_sched(r);
  LM_DISPATCH_N(r->d.N, lm::launch_prologue, *r);
  if ((s = check_launch()) != LM_OK) return s;
  r->n_tau = r->n;
  r->in_interval = true;
  return LM_OK;
}

lm_status lm_step(lm_run* r, int32_t nsteps) {
  if (!r) return fail(LM_E_ARG, "null run");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  if (nsteps < 0) return fail(LM_E_ARG, "nsteps < 0");
  if (!r->has_state) return fail(LM_E_STATE, "no state set");
  use_sched(r);
  LM_DISPATCH_N(r->d.N, lm::launch_steps, *r, nsteps);
  return check_launch();
}

lm_status lm_step_timed(lm_run* r, int32_t nsteps, double* ms) {
  if (!r || !ms) return fail(LM_E_ARG, "null argument");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  if (nsteps < 0) return fail(LM_E_ARG, "nsteps < 0");
  if (!r->has_state) return fail(LM_E_STATE, "no state set");
  const StreamDrain drain{r->stream};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, r->stream);
  if (e == hipSuccess) {
    use_sched(r);
    LM_DISPATCH_N(r->d.N, lm::launch_steps, *r, nsteps);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, r->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(LM_E_HIP, std::string("timed steps: ") + hipGetErrorString(e));
  *ms = t;
  return LM_OK;
}

lm_status lm_step_profiled(lm_run* r, int32_t nsteps, double* ms_avg) {
  if (!r || !ms_avg) return fail(LM_E_ARG, "null argument");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  if (nsteps <= 0 || nsteps > 4096) return fail(LM_E_ARG, "nsteps must be in 1..4096");
  if (!r->has_state) return fail(LM_E_STATE, "no state set");
  double ms[3] = {0.0, 0.0, 0.0};
  hipError_t e = hipSuccess;
  use_sched(r);
  LM_DISPATCH_N_RET(r->d.N, e, lm::launch_steps_profiled, *r, nsteps, ms);
  if (e != hipSuccess) return fail(LM_E_HIP, std::string("profiled step: ") + hipGetErrorString(e));
  lm_status s = check_launch();
  if (s != LM_OK) return s;
  for (int i = 0; i < 3; ++i) ms_avg[i] = ms[i] / (4.0 * nsteps);
  return LM_OK;
}

lm_status lm_end_interval(lm_run* r, double* T_out) {
  if (!r) return fail(LM_E_ARG, "null run");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  if (!r->in_interval) return fail(LM_E_STATE, "no open interval");
  if (r->n == r->n_tau) return fail(LM_E_STATE, "interval holds no step");
  const double T = double(r->n - r->n_tau) * r->ph.dt;
  const StreamDrain drain{r->stream};
  const size_t nn = (size_t)r->d.N * r->d.N, rf = r->d.rowfield_elems();
  cplx<double>* ioC = (cplx<double>*)r->at(r->L.ioC);
  double* out = (double*)r->at(r->L.out);
  r->has_remap = false;  // a remap describes the previous outputs
  // accumulators in output order: (gbar_h, gbar_z), (xi_x, xi_y), (gtil_h, gtil_z), (P_x, P_y), (E_h, E_z)
  static const int order[10] = {LM_P_GBAR_H, LM_P_GBAR_ZETA, LM_P_XI_X, LM_P_XI_Y, LM_P_GTIL_H,
                                LM_P_GTIL_ZETA, LM_P_P_X, LM_P_P_Y, LM_P_E_H, LM_P_E_ZETA};
  for (int half = 0; half < 2; ++half) {
    lm::IoColInv J{};
    for (int q = 0; q < 5; ++q) {
      const FieldRef f = state_field(r, order[half * 5 + q]);
      J.src[q] = f.ptr;
      J.src_lo[q] = f.lo;
      J.src_f32[q] = f.f32;
      J.dst[q] = ioC + (half * 5 + q) * rf;
    }
    LM_DISPATCH_N(r->d.N, lm::launch_io_col_inverse, *r, J, 5);
  }
  lm::IoRowInv K{};
  for (int p = 0; p < 5; ++p) {
    K.a[p] = ioC + (2 * p) * rf;
    K.b[p] = ioC + (2 * p + 1) * rf;
    K.oa[p] = out + (2 * p) * nn;
    K.ob[p] = out + (2 * p + 1) * nn;
    const double sc = (p == 1) ? 1.0 : 1.0 / T;  // xi is not divided
    K.sa[p] = K.sb[p] = sc;
    // the h accumulators integrate eta = h - H: the mean of h is H + (mean of eta)
    // (h, when averaged, is always the first field)
    K.ca[p] = ((p == 0 || p == 2 || p == 4) && r->ph.fs0 == lm::FS_ETA) ? r->ph.H : 0.0;
    K.cb[p] = 0.0;
  }
  LM_DISPATCH_N(r->d.N, lm::launch_io_row_inverse, *r, K, 5);
  if (r->mom) {
    // the momentum 1-form mean g-bar_m / T (planes OUT_MOM, OUT_MOM + 1)
    lm::IoColInv Jm{};
    for (int q = 0; q < 2; ++q) {
      const FieldRef f = real_field(r, lm::SF_GMX + q);
      Jm.src[q] = f.ptr;
      Jm.src_lo[q] = f.lo;
      Jm.src_f32[q] = f.f32;
      Jm.dst[q] = ioC + q * rf;
    }
    LM_DISPATCH_N(r->d.N, lm::launch_io_col_inverse, *r, Jm, 2);
    lm::IoRowInv Km{};
    Km.a[0] = ioC;
    Km.b[0] = ioC + rf;
    Km.oa[0] = out + lm::OUT_MOM * nn;
    Km.ob[0] = out + (lm::OUT_MOM + 1) * nn;
    Km.sa[0] = Km.sb[0] = 1.0 / T;
    LM_DISPATCH_N(r->d.N, lm::launch_io_row_inverse, *r, Km, 1);
  }
  int* flag = (int*)r->at(r->L.flag);
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), r->stream));
  lm::launch_nonfinite(*r, out, 10 * nn, flag);
  if (r->mom) lm::launch_nonfinite(*r, out + lm::OUT_MOM * nn, 2 * nn, flag);
  lm_status s;
  if ((s = check_launch()) != LM_OK) return s;
  // the flag is read with a blocking copy once the stream has drained
  int hflag = 0;
  HIP_TRY(hipStreamSynchronize(r->stream));
  HIP_TRY(hipMemcpy(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost));
  r->T = T;
  r->has_mean = true;
  r->in_interval = false;
  if (T_out) *T_out = T;
  if (hflag) return fail(LM_E_NONFINITE, "non-finite values in the interval outputs");
  return LM_OK;
}

lm_status lm_remap_s1(lm_run* r, int32_t max_extent, double* residual) {
  if (!r) return fail(LM_E_ARG, "null run");
  if (max_extent < 1 || max_extent > 64) return fail(LM_E_ARG, "max_extent must be in 1..64");
  if (!r->has_mean) return fail(LM_E_STATE, "no closed interval");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  const StreamDrain drain{r->stream};
  const size_t nn = (size_t)r->d.N * r->d.N;
  double* out = (double*)r->at(r->L.out);
  unsigned long long* bits = (unsigned long long*)r->at(r->L.resid);
  // the boundary staging buffer (3 N^2 float64) holds the claims (N^2 uint32)
  unsigned* best = (unsigned*)r->at(r->L.phys);
  HIP_TRY(hipMemsetAsync(bits, 0, sizeof(unsigned long long), r->stream));
  // inputs: S1 means (planes 4, 5) and eta (6, 7); outputs after the Eulerian planes
  lm::launch_remap_s1(*r, out + 4 * nn, out + 5 * nn, out + 6 * nn, out + 7 * nn, out + lm::OUT_REMAP * nn, best,
                      max_extent, bits);
  lm_status s;
  if ((s = check_launch()) != LM_OK) return s;
  unsigned long long hb = 0;
  HIP_TRY(hipStreamSynchronize(r->stream));
  HIP_TRY(hipMemcpy(&hb, bits, sizeof(hb), hipMemcpyDeviceToHost));
  double res;
  memcpy(&res, &hb, sizeof(res));
  r->has_remap = true;
  if (residual) *residual = res;
  return LM_OK;
}

lm_status lm_read_mean(lm_run* r, int32_t field, int32_t kind, double* out_, int on_device) {
  if (!r || !out_) return fail(LM_E_ARG, "null argument");
  if (!r->has_mean) return fail(LM_E_STATE, "no closed interval");
  if (field != LM_FIELD_H && field != LM_FIELD_ZETA) return fail(LM_E_ARG, "field must be LM_FIELD_H or LM_FIELD_ZETA");
  int idx;
  switch (kind) {
    case LM_K_S2_MEAN: idx = 0 + field; break;
    case LM_K_S2_XI_X: idx = 2; break;
    case LM_K_S2_XI_Y: idx = 3; break;
    case LM_K_S1_MEAN: idx = 4 + field; break;
    case LM_K_S1_ETA_X: idx = 6; break;
    case LM_K_S1_ETA_Y: idx = 7; break;
    case LM_K_EULER_MEAN: idx = 8 + field; break;
    case LM_K_S1_REMAP_MEAN: idx = lm::OUT_REMAP + field; break;
    case LM_K_S1_REMAP_XI_X: idx = lm::OUT_REMAP + 2; break;
    case LM_K_S1_REMAP_XI_Y: idx = lm::OUT_REMAP + 3; break;
    case LM_K_S2_MOM_X: idx = lm::OUT_MOM; break;
    case LM_K_S2_MOM_Y: idx = lm::OUT_MOM + 1; break;
    default: return fail(LM_E_ARG, "unknown kind");
  }
  if (idx >= lm::OUT_MOM && !r->mom) return fail(LM_E_STATE, "the run does not average the momentum 1-form");
  if (idx >= lm::OUT_REMAP && idx < lm::OUT_REMAP + 4 && !r->has_remap)
    return fail(LM_E_STATE, "no strategy-1 remap of the last interval");
  const StreamDrain drain{r->stream};
  const size_t nn = (size_t)r->d.N * r->d.N;
  lm_status s = copy_out(r, out_, (double*)r->at(r->L.out) + idx * nn, on_device);
  if (s != LM_OK) return s;
  HIP_TRY(hipStreamSynchronize(r->stream));
  return LM_OK;
}

lm_status lm_peek(lm_run* r, int32_t which, double* out_, int on_device) {
  if (!r || !out_) return fail(LM_E_ARG, "null argument");
  if (which < LM_P_U || which > LM_P_P_Y) return fail(LM_E_ARG, "unknown field");
  if (!r->has_state) return fail(LM_E_STATE, "no state set");
  const StreamDrain drain{r->stream};
  cplx<double>* ioC = (cplx<double>*)r->at(r->L.ioC);
  double* phys = (double*)r->at(r->L.phys);
  lm::IoColInv J{};
  const FieldRef f = state_field(r, which);
  J.src[0] = f.ptr;
  J.src_lo[0] = f.lo;
  J.src_f32[0] = f.f32;
  J.dst[0] = ioC;
  LM_DISPATCH_N(r->d.N, lm::launch_io_col_inverse, *r, J, 1);
  lm::IoRowInv K{};
  K.a[0] = ioC; K.b[0] = nullptr; K.oa[0] = phys; K.ob[0] = nullptr; K.sa[0] = 1.0;
  LM_DISPATCH_N(r->d.N, lm::launch_io_row_inverse, *r, K, 1);
  lm_status s;
  if ((s = check_launch()) != LM_OK) return s;
  if ((s = copy_out(r, out_, phys, on_device)) != LM_OK) return s;
  HIP_TRY(hipStreamSynchronize(r->stream));
  return LM_OK;
}

}  // extern "C"

namespace {

// checkpoint layout: this header, then the working-precision state (leading
// words), its trailing words (float runs) and the float64 state, as stored
struct CkHeader {
  char magic[8];
  int32_t n, precision, interp, mode, mom, gen, fs0, fs1;
  double f, g, H, dt, nu8, kin[7];
  int64_t steps, n_tau;
  int32_t in_interval, reserved;
  uint64_t bytes_r, bytes_l, bytes_d;
};
constexpr char CK_MAGIC[8] = {'L', 'M', 'C', 'K', 'P', 'T', '0', '1'};

CkHeader ck_header(const lm_run* r) {
  CkHeader h{};
  memcpy(h.magic, CK_MAGIC, 8);
  h.n = r->d.N;
  h.precision = r->fp32 ? LM_FP32_MIXED : LM_FP64;
  h.interp = r->cfg.interp;
  h.mode = r->cfg.mode;
  h.mom = r->ph.mom;
  h.gen = r->ph.gen;
  h.fs0 = r->ph.fs0;
  h.fs1 = r->ph.fs1;
  h.f = r->ph.f;
  h.g = r->ph.g;
  h.H = r->ph.H;
  h.dt = r->ph.dt;
  h.nu8 = r->ph.nu8;
  const double kin[7] = {r->ph.kx, r->ph.ky, r->ph.A, r->ph.omega, r->ph.phase, r->ph.U0, r->ph.V0};
  memcpy(h.kin, kin, sizeof(kin));
  h.steps = r->n;
  h.n_tau = r->n_tau;
  h.in_interval = r->in_interval ? 1 : 0;
  const size_t sp = r->d.spec_elems();
  const size_t cT = r->fp32 ? sizeof(cplx<float>) : sizeof(cplx<double>);
  const int nsf = r->mom ? lm::NSF_R : lm::SF_GMX;
  h.bytes_r = nsf * sp * cT;
  h.bytes_l = r->fp32 ? h.bytes_r : 0;
  h.bytes_d = lm::NSF_D * sp * sizeof(cplx<double>);
  return h;
}

size_t ck_size(const CkHeader& h) { return sizeof(CkHeader) + h.bytes_r + h.bytes_l + h.bytes_d; }

}  // namespace

extern "C" {

lm_status lm_checkpoint_size(const lm_run* r, size_t* bytes) {
  if (!r || !bytes) return fail(LM_E_ARG, "null argument");
  *bytes = ck_size(ck_header(r));
  return LM_OK;
}

lm_status lm_save(lm_run* r, void* buf, size_t cap, int on_device) {
  if (!r || !buf) return fail(LM_E_ARG, "null argument");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  if (!r->has_state) return fail(LM_E_STATE, "no state set");
  const CkHeader h = ck_header(r);
  if (cap < ck_size(h)) return fail(LM_E_ARG, "buffer smaller than lm_checkpoint_size");
  const StreamDrain drain{r->stream};  // every copy has landed before any return
  const hipMemcpyKind d2x = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  char* out = (char*)buf;
  if (on_device) HIP_TRY(hipMemcpyAsync(out, &h, sizeof(h), hipMemcpyHostToDevice, r->stream));
  else memcpy(out, &h, sizeof(h));
  size_t off = sizeof(h);
  HIP_TRY(hipMemcpyAsync(out + off, r->slab + r->L.Yr, h.bytes_r, d2x, r->stream));
  off += h.bytes_r;
  if (h.bytes_l) HIP_TRY(hipMemcpyAsync(out + off, r->slab + r->L.Yl, h.bytes_l, d2x, r->stream));
  off += h.bytes_l;
  HIP_TRY(hipMemcpyAsync(out + off, r->slab + r->L.Yd, h.bytes_d, d2x, r->stream));
  HIP_TRY(hipStreamSynchronize(r->stream));
  return LM_OK;
}

lm_status lm_restore(lm_run* r, const void* buf, size_t size, int on_device) {
  if (!r || !buf) return fail(LM_E_ARG, "null argument");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  const StreamDrain drain{r->stream};
  CkHeader h{};
  if (size < sizeof(h)) return fail(LM_E_ARG, "not a checkpoint (too short)");
  if (on_device) HIP_TRY(hipMemcpy(&h, buf, sizeof(h), hipMemcpyDeviceToHost));
  else memcpy(&h, buf, sizeof(h));
  const CkHeader mine = ck_header(r);
  if (memcmp(h.magic, CK_MAGIC, 8) != 0) return fail(LM_E_ARG, "not a checkpoint of this library");
  // the configuration must be the run's own, field for field
  if (h.n != mine.n || h.precision != mine.precision || h.interp != mine.interp || h.mode != mine.mode ||
      h.mom != mine.mom || h.gen != mine.gen || h.fs0 != mine.fs0 || h.fs1 != mine.fs1 ||
      memcmp(&h.f, &mine.f, 5 * sizeof(double)) != 0 || memcmp(h.kin, mine.kin, sizeof(h.kin)) != 0 ||
      h.bytes_r != mine.bytes_r || h.bytes_l != mine.bytes_l || h.bytes_d != mine.bytes_d)
    return fail(LM_E_ARG, "the checkpoint was taken with another configuration");
  if (size < ck_size(h)) return fail(LM_E_ARG, "checkpoint truncated");
  if (h.steps < 0 || h.n_tau < 0 || h.n_tau > h.steps) return fail(LM_E_ARG, "checkpoint counters out of range");
  const hipMemcpyKind x2d = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  const char* in = (const char*)buf;
  size_t off = sizeof(h);
  HIP_TRY(hipMemcpyAsync(r->slab + r->L.Yr, in + off, h.bytes_r, x2d, r->stream));
  off += h.bytes_r;
  if (h.bytes_l) HIP_TRY(hipMemcpyAsync(r->slab + r->L.Yl, in + off, h.bytes_l, x2d, r->stream));
  off += h.bytes_l;
  HIP_TRY(hipMemcpyAsync(r->slab + r->L.Yd, in + off, h.bytes_d, x2d, r->stream));
  r->n = h.steps;
  r->n_tau = h.n_tau;
  r->ys_cur = 0;
  // the column-pass outputs and stage values of the current state, as the last
  // step's final column pass left them
  use_sched(r);
  LM_DISPATCH_N(r->d.N, lm::launch_prologue, *r);
  lm_status s;
  if ((s = check_launch()) != LM_OK) return s;
  HIP_TRY(hipStreamSynchronize(r->stream));
  r->has_state = true;
  r->in_interval = h.in_interval != 0;
  r->has_mean = r->has_remap = false;
  return LM_OK;
}

lm_status lm_counters(lm_run* r, int64_t* steps, int64_t* steps_in_interval) {
  if (!r) return fail(LM_E_ARG, "null run");
  if (steps) *steps = r->n;
  if (steps_in_interval) *steps_in_interval = r->in_interval ? r->n - r->n_tau : 0;
  return LM_OK;
}

lm_status lm_destroy(lm_run* r) {
  if (!r) return LM_OK;
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  hipError_t e = hipStreamSynchronize(r->stream);
  release_streams(r);
  hipError_t e2 = hipFree(r->slab);
  delete r;
  if (e != hipSuccess) return fail(LM_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(LM_E_HIP, std::string("hipFree: ") + hipGetErrorString(e2));
  return LM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
namespace {

lm_batch::Group* batch_group(lm_batch* b, int N, bool fp32, bool cubic, bool mom, bool gen) {
  for (auto& g : b->groups)
    if (g.N == N && g.fp32 == fp32 && g.cubic == cubic && g.mom == mom && g.gen == gen) return &g;
  lm_batch::Group g;
  g.N = N;
  g.fp32 = fp32;
  g.cubic = cubic;
  g.mom = mom;
  g.gen = gen;
  if (hipStreamCreateWithFlags(&g.fork, hipStreamNonBlocking) != hipSuccess) return nullptr;
  if (hipEventCreateWithFlags(&g.join, hipEventDisableTiming) != hipSuccess) return nullptr;
  b->groups.push_back(g);
  return &b->groups.back();
}

template <typename T>
std::vector<char> group_descs(lm_batch* b, const lm_batch::Group& g, const std::vector<int>& active, int* count) {
  std::vector<lm::RunDesc<T>> d;
  for (int i : active) {
    lm_run* r = b->members[i].run;
    if (r->d.N == g.N && r->fp32 == g.fp32 && r->cubic == g.cubic && r->mom == g.mom && (bool)r->ph.gen == g.gen)
      d.push_back(lm::run_desc<T>(*r, b->d_counters + i));
  }
  *count = (int)d.size();
  std::vector<char> bytes(d.size() * sizeof(lm::RunDesc<T>));
  if (!d.empty()) memcpy(bytes.data(), d.data(), bytes.size());
  return bytes;
}

void drop_graph(lm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->signature.clear();
}

// descriptors of the active members, then one captured graph for one RK4 step
lm_status batch_rebuild(lm_batch* b, const std::vector<int>& active) {
  // steps already queued read the descriptor arrays rewritten below (and run
  // the graph destroyed here): they must have finished first
  HIP_TRY(hipStreamSynchronize(b->stream));
  drop_graph(b);
  struct Launch {
    lm_batch::Group* g;
    int count;
  };
  std::vector<Launch> launches;
  for (int i : active) {
    lm_run* r = b->members[i].run;
    lm_batch::Group* g = batch_group(b, r->d.N, r->fp32, r->cubic, r->mom, r->ph.gen);
    if (!g) return fail(LM_E_HIP, "batch: stream or event creation failed");
  }
  for (auto& g : b->groups) {
    int count = 0;
    std::vector<char> bytes = g.fp32 ? group_descs<float>(b, g, active, &count)
                                     : group_descs<double>(b, g, active, &count);
    if (count == 0) continue;
    if (bytes.size() > g.cap) {
      if (g.d_desc) (void)hipFree(g.d_desc);
      g.d_desc = nullptr;
      g.cap = 0;
      if (hipMalloc(&g.d_desc, bytes.size()) != hipSuccess) return fail(LM_E_OOM, "batch: descriptor allocation");
      g.cap = bytes.size();
    }
    HIP_TRY(hipMemcpy(g.d_desc, bytes.data(), bytes.size(), hipMemcpyHostToDevice));
    launches.push_back({&g, count});
  }
  std::vector<lm::Sched> scheds;
  unsigned gen = sched_gen();
  for (auto& l : launches) scheds.push_back(get_sched(l.g->N, l.g->fp32, true, &gen));
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  // from here on the capture is always ended, whatever fails
  hipError_t e = hipEventRecord(b->fork_ev, b->stream);
  for (size_t li = 0; li < launches.size(); ++li) {
    const Launch& l = launches[li];
    if (e == hipSuccess) e = hipStreamWaitEvent(l.g->fork, b->fork_ev, 0);
    if (e == hipSuccess) {
      lm::Phys gp{};
      gp.mom = l.g->mom;
      gp.gen = l.g->gen;
      LM_DISPATCH_N(l.g->N, lm::launch_batch_step, l.g->fork, l.g->d_desc, l.count, l.g->fp32, l.g->cubic, l.g->mom,
                    lm::col_groups(gp), scheds[li]);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(l.g->join, l.g->fork);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, l.g->join, 0);
  }
  if (e == hipSuccess) {
    lm::launch_batch_tick(b->stream, b->d_counters, (int)b->members.size());
    e = hipGetLastError();
  }
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(LM_E_HIP, std::string("batch capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  }
  b->graph = graph;
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return fail(LM_E_HIP, std::string("batch graph: ") + hipGetErrorString(e));
  }
  for (int i : active) b->signature.push_back(b->members[i].run);
  b->sched_gen = gen;
  return LM_OK;
}

int find_member(const lm_batch* b, const lm_run* r) {
  for (size_t i = 0; i < b->members.size(); ++i)
    if (b->members[i].run == r) return (int)i;
  return -1;
}

}  // namespace

extern "C" {

lm_status lm_batch_create(void* hip_stream, lm_batch** out) {
  if (!out) return fail(LM_E_ARG, "null out");
  lm_batch* b = new lm_batch();
  b->user = (hipStream_t)hip_stream;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(LM_E_HIP, "batch: stream creation failed");
  }
  if (hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(b->stream);
    delete b;
    return fail(LM_E_HIP, "batch: event creation failed");
  }
  *out = b;
  return LM_OK;
}

lm_status lm_batch_add(lm_batch* b, lm_run* r, int32_t steps) {
  if (!b || !r) return fail(LM_E_ARG, "null argument");
  if (steps < 0) return fail(LM_E_ARG, "steps < 0");
  if (r->batch) return fail(LM_E_STATE, "the run already belongs to a batch");
  if (!r->has_state || !r->in_interval) return fail(LM_E_STATE, "the run needs a state and an open interval");
  HIP_TRY(hipStreamSynchronize(r->stream));
  b->members.push_back({r, steps});
  r->batch = b;
  drop_graph(b);
  return LM_OK;
}

lm_status lm_batch_remove(lm_batch* b, lm_run* r) {
  if (!b || !r) return fail(LM_E_ARG, "null argument");
  const int i = find_member(b, r);
  if (i < 0) return fail(LM_E_ARG, "not a member");
  // no queued batch step may still write the run's buffers once it has left
  const hipError_t e = hipStreamSynchronize(b->stream);
  b->members.erase(b->members.begin() + i);
  r->batch = nullptr;
  drop_graph(b);
  if (e != hipSuccess) return fail(LM_E_HIP, std::string("batch remove: ") + hipGetErrorString(e));
  return LM_OK;
}

lm_status lm_batch_remaining(lm_batch* b, const lm_run* r, int32_t* remaining) {
  if (!b || !r || !remaining) return fail(LM_E_ARG, "null argument");
  const int i = find_member(b, r);
  if (i < 0) return fail(LM_E_ARG, "not a member");
  *remaining = b->members[i].remaining;
  return LM_OK;
}

}  // extern "C"

namespace {

// device step counters for the members (allocated on first use, grown with
// the batch), after the caller's stream and the members' own streams: their
// values from the host counters
lm_status upload_counters(lm_batch* b) {
  const int m = (int)b->members.size();
  if (m > b->counter_cap) {
    if (b->d_counters) (void)hipFree(b->d_counters);
    b->d_counters = nullptr;
    b->counter_cap = 0;
    const int cap = std::max(64, 2 * m);
    if (hipMalloc((void**)&b->d_counters, cap * sizeof(long long)) != hipSuccess)
      return fail(LM_E_OOM, "batch: counter allocation");
    b->counter_cap = cap;
    drop_graph(b);  // descriptors point into the counter array
  }
  // the caller's stream and the members' own streams first; then the device
  // step counters from the host ones
  HIP_TRY(hipStreamSynchronize(b->user));
  std::vector<long long> cnt(m);
  for (int i = 0; i < m; ++i) {
    HIP_TRY(hipStreamSynchronize(b->members[i].run->stream));
    cnt[i] = b->members[i].run->n - b->members[i].run->n_tau;
  }
  if (m > 0) HIP_TRY(hipMemcpy(b->d_counters, cnt.data(), m * sizeof(long long), hipMemcpyHostToDevice));
  (void)hipGetLastError();
  return LM_OK;
}

}  // namespace

extern "C" {

lm_status lm_batch_step(lm_batch* b, int32_t max_steps, int32_t* active_out) {
  if (!b) return fail(LM_E_ARG, "null batch");
  if (max_steps < 0) return fail(LM_E_ARG, "max_steps < 0");
  const StreamDrain drain{b->stream};  // every path out leaves no batch step in flight
  const int m = (int)b->members.size();
  lm_status st = upload_counters(b);
  if (st != LM_OK) return st;
  for (int it = 0; it < max_steps; ++it) {
    std::vector<int> active;
    for (int i = 0; i < m; ++i)
      if (b->members[i].remaining > 0) active.push_back(i);
    if (active.empty()) break;
    bool same = b->exec && active.size() == b->signature.size() && b->sched_gen == sched_gen();
    for (size_t j = 0; same && j < active.size(); ++j) same = b->members[active[j]].run == b->signature[j];
    if (!same) {
      lm_status s = batch_rebuild(b, active);
      if (s != LM_OK) return s;
    }
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    for (int i : active) {
      b->members[i].remaining -= 1;
      b->members[i].run->n += 1;
    }
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (active_out) {
    int a = 0;
    for (auto& mm : b->members) a += mm.remaining > 0;
    *active_out = a;
  }
  return LM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free batched step
// ---------------------------------------------------------------------------
namespace {

// Device scratch of lm_batch_step_static, one copy per GPU for the life of the
// process: the step counters of up to LM_STATIC_MAX_MEMBERS members (first
// 2 KiB), then the run descriptors of each (N, precision, gathers, momentum,
// fields) group, packed, each group's array 256-byte aligned.  In host code
// `scratch` names a host-side stand-in: kernels and copies get the device
// address from static_scratch() instead.
constexpr size_t STATIC_BYTES = 128 * 1024;
constexpr size_t STATIC_COUNTERS = LM_STATIC_MAX_MEMBERS * sizeof(long long);
static_assert(STATIC_COUNTERS + LM_STATIC_MAX_MEMBERS * (sizeof(lm::RunDesc<double>) + 256) <= STATIC_BYTES,
              "static scratch too small for its member limit");
static_assert(sizeof(lm::RunDesc<float>) <= sizeof(lm::RunDesc<double>), "descriptor sizes");
__device__ __align__(256) unsigned char scratch[STATIC_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};  // device address of scratch, per device ordinal

// the calling thread's current device's copy of scratch (looked up once per device)
lm_status static_scratch(unsigned char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(LM_E_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LM_E_HIP, "hipGetSymbolAddress returned a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = (unsigned char*)g_scratch_ptr[dev];
  return LM_OK;
}

struct StaticGroup {
  int N;
  bool fp32, cubic, mom, gen;
  int count;
  size_t off;  // byte offset of its descriptor array in scratch
};

bool same_group(const StaticGroup& g, const lm_run* r) {
  return g.N == r->d.N && g.fp32 == r->fp32 && g.cubic == r->cubic && g.mom == r->mom && g.gen == (bool)r->ph.gen;
}

}  // namespace

extern "C" {

lm_status lm_batch_step_static(lm_batch* b, int32_t max_steps, int32_t* active_out) {
  if (!b) return fail(LM_E_ARG, "null batch");
  if (max_steps < 0) return fail(LM_E_ARG, "max_steps < 0");
  const int m = (int)b->members.size();
  if (m > LM_STATIC_MAX_MEMBERS)
    return fail(LM_E_BUDGET, "lm_batch_step_static: the batch has " + std::to_string(m) +
                                 " members, more than LM_STATIC_MAX_MEMBERS (" +
                                 std::to_string(LM_STATIC_MAX_MEMBERS) + ")");
  unsigned char* dev = nullptr;
  lm_status st = static_scratch(&dev);
  if (st != LM_OK) return st;
  const StreamDrain drain{b->stream};  // every path out leaves no step in flight
  // the caller's stream and the members' own streams first
  HIP_TRY(hipStreamSynchronize(b->user));
  for (int i = 0; i < m; ++i) HIP_TRY(hipStreamSynchronize(b->members[i].run->stream));
  // the batch's own stream too: earlier steps read the scratch rewritten below
  HIP_TRY(hipStreamSynchronize(b->stream));
  unsigned char* stage = b->static_stage;
  long long* cnt = reinterpret_cast<long long*>(stage);
  for (int i = 0; i < m; ++i) cnt[i] = b->members[i].run->n - b->members[i].run->n_tau;
  if (m > 0) HIP_TRY(hipMemcpyAsync(dev, stage, m * sizeof(long long), hipMemcpyHostToDevice, b->stream));
  long long* d_cnt = reinterpret_cast<long long*>(dev);

  int active[LM_STATIC_MAX_MEMBERS];
  int nact_prev = -1;
  StaticGroup groups[LM_STATIC_MAX_MEMBERS];
  int ngroups = 0;
  for (int it = 0; it < max_steps; ++it) {
    int nact = 0;
    for (int i = 0; i < m; ++i)
      if (b->members[i].remaining > 0) active[nact++] = i;
    if (nact == 0) break;
    if (nact != nact_prev) {
      // the active set changed (members only drop out): new descriptors, after
      // the queued steps that read the old ones
      HIP_TRY(hipStreamSynchronize(b->stream));
      ngroups = 0;
      for (int a = 0; a < nact; ++a) {
        const lm_run* r = b->members[active[a]].run;
        int g = 0;
        while (g < ngroups && !same_group(groups[g], r)) ++g;
        if (g == ngroups) groups[ngroups++] = {r->d.N, r->fp32, r->cubic, r->mom, (bool)r->ph.gen, 0, 0};
        groups[g].count += 1;
      }
      size_t off = STATIC_COUNTERS;
      for (int g = 0; g < ngroups; ++g) {
        groups[g].off = off;
        int k = 0;
        for (int a = 0; a < nact; ++a) {
          lm_run* r = b->members[active[a]].run;
          if (!same_group(groups[g], r)) continue;
          if (r->fp32) {
            const lm::RunDesc<float> d = lm::run_desc<float>(*r, d_cnt + active[a]);
            memcpy(stage + off + k * sizeof(d), &d, sizeof(d));
          } else {
            const lm::RunDesc<double> d = lm::run_desc<double>(*r, d_cnt + active[a]);
            memcpy(stage + off + k * sizeof(d), &d, sizeof(d));
          }
          ++k;
        }
        off += (groups[g].count * sizeof(lm::RunDesc<double>) + 255) / 256 * 256;
      }
      HIP_TRY(hipMemcpyAsync(dev + STATIC_COUNTERS, stage + STATIC_COUNTERS, off - STATIC_COUNTERS,
                             hipMemcpyHostToDevice, b->stream));
      nact_prev = nact;
    }
    // one RK4 step of every group, launched directly on the batch's stream
    for (int g = 0; g < ngroups; ++g) {
      lm::Phys gp{};
      gp.mom = groups[g].mom;
      gp.gen = groups[g].gen;
      const lm::Sched sc = get_sched(groups[g].N, groups[g].fp32, true);
      LM_DISPATCH_N(groups[g].N, lm::launch_batch_step, b->stream, dev + groups[g].off, groups[g].count,
                    groups[g].fp32, groups[g].cubic, groups[g].mom, lm::col_groups(gp), sc);
    }
    lm::launch_batch_tick(b->stream, d_cnt, m);
    st = check_launch();
    if (st != LM_OK) return st;
    for (int a = 0; a < nact; ++a) {
      b->members[active[a]].remaining -= 1;
      b->members[active[a]].run->n += 1;
    }
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (active_out) {
    int a = 0;
    for (auto& mm : b->members) a += mm.remaining > 0;
    *active_out = a;
  }
  return LM_OK;
}

lm_status lm_batch_autotune(lm_batch* b, int32_t steps, int32_t reps, int32_t* tuned) {
  if (!b) return fail(LM_E_ARG, "null batch");
  if (steps < 1 || steps > 64) return fail(LM_E_ARG, "steps must be in 1..64");
  if (reps < 1 || reps > 16) return fail(LM_E_ARG, "reps must be in 1..16");
  const int m = (int)b->members.size();
  if (tuned) *tuned = 0;
  if (m == 0) return LM_OK;
  lm_status st = upload_counters(b);  // also waits for every stream that may touch the members
  if (st != LM_OK) return st;
  // a copy of every member's allocation and host counters
  std::vector<void*> snap(m, nullptr);
  std::vector<int64_t> n0(m), nt0(m);
  std::vector<int> ys0(m);
  hipError_t e = hipSuccess;
  for (int i = 0; i < m && e == hipSuccess; ++i) {
    lm_run* r = b->members[i].run;
    n0[i] = r->n;
    nt0[i] = r->n_tau;
    ys0[i] = r->ys_cur;
    e = hipMalloc(&snap[i], r->L.total);
    if (e == hipSuccess) e = hipMemcpyAsync(snap[i], r->slab, r->L.total, hipMemcpyDeviceToDevice, b->stream);
  }
  const bool have_copy = (e == hipSuccess);
  auto restore = [&]() -> hipError_t {
    hipError_t x = hipSuccess;
    for (int i = 0; i < m && x == hipSuccess; ++i) {
      lm_run* r = b->members[i].run;
      r->n = n0[i];
      r->n_tau = nt0[i];
      r->ys_cur = ys0[i];
      if (have_copy) x = hipMemcpyAsync(r->slab, snap[i], r->L.total, hipMemcpyDeviceToDevice, b->stream);
    }
    return x;
  };
  // (N, precision) keys present, each tuned in turn with the others at their current schedule
  std::vector<std::pair<int, bool>> keys;
  for (auto& mm : b->members) {
    const std::pair<int, bool> k{mm.run->d.N, mm.run->fp32};
    if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
  }
  std::vector<int> all(m);
  for (int i = 0; i < m; ++i) all[i] = i;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  lm_status ls = LM_OK;
  for (size_t ki = 0; ki < keys.size() && e == hipSuccess && ls == LM_OK; ++ki) {
    const int N = keys[ki].first;
    const bool fp32 = keys[ki].second;
    const std::vector<lm::Sched> cand = sched_candidates(N, fp32, true);
    lm::Sched best = get_sched(N, fp32, true);
    double best_t = -1.0;
    for (size_t c = 0; c < cand.size() && e == hipSuccess && ls == LM_OK; ++c) {
      put_sched(N, fp32, true, cand[c]);
      ls = batch_rebuild(b, all);
      double bt = -1.0;
      for (int rep = 0; rep < reps && e == hipSuccess && ls == LM_OK; ++rep) {
        e = restore();
        // the graph's tick advances the device counters: start every trial from the host ones
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e == hipSuccess) ls = upload_counters(b);
        if (e == hipSuccess && ls == LM_OK) e = hipEventRecord(e0, b->stream);
        for (int s = 0; s < steps && e == hipSuccess && ls == LM_OK; ++s) e = hipGraphLaunch(b->exec, b->stream);
        if (e == hipSuccess && ls == LM_OK) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess && ls == LM_OK) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess && ls == LM_OK) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess && ls == LM_OK && (bt < 0.0 || t < bt)) bt = t;
      }
      if (e == hipSuccess && ls == LM_OK && (best_t < 0.0 || bt < best_t)) {
        best_t = bt;
        best = cand[c];
      }
    }
    put_sched(N, fp32, true, best);
  }
  // the members as they were, their device counters from the host ones, and
  // a graph captured afresh at the next lm_batch_step
  const hipError_t er = restore();
  const hipError_t es = hipStreamSynchronize(b->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void* p : snap)
    if (p) (void)hipFree(p);
  drop_graph(b);
  if (ls != LM_OK) return ls;
  if (e == hipSuccess) e = (er != hipSuccess) ? er : es;
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? LM_E_OOM : LM_E_HIP, std::string("batch autotune: ") + hipGetErrorString(e));
  }
  st = upload_counters(b);
  if (st != LM_OK) return st;
  if (tuned) *tuned = (int32_t)keys.size();
  return LM_OK;
}

// ---------------------------------------------------------------------------
// launch schedules and the autotuner
// ---------------------------------------------------------------------------

lm_status lm_schedule_candidates(int32_t n, int32_t precision, lm_schedule* out, int32_t cap, int32_t* count) {
  if (!supported_n(n)) return fail(LM_E_UNSUPPORTED, "n must be 64, 128, 192, 256, 384, 512 or 1024");
  if (precision != LM_FP64 && precision != LM_FP32_MIXED) return fail(LM_E_ARG, "unknown precision");
  if (cap < 0 || (cap > 0 && !out)) return fail(LM_E_ARG, "cap < 0 or null out");
  const std::vector<lm::Sched> c = sched_candidates(n, precision == LM_FP32_MIXED);
  for (int i = 0; i < (int)c.size() && i < cap; ++i) out[i] = lm_schedule{c[i].tile, c[i].remap, c[i].streams};
  if (count) *count = (int32_t)c.size();
  return LM_OK;
}

}  // extern "C"

namespace {

lm_status set_schedule_ctx(int32_t n, int32_t precision, const lm_schedule* s, bool batched) {
  if (!supported_n(n)) return fail(LM_E_UNSUPPORTED, "n must be 64, 128, 192, 256, 384, 512 or 1024");
  if (precision != LM_FP64 && precision != LM_FP32_MIXED) return fail(LM_E_ARG, "unknown precision");
  if (!s) return fail(LM_E_ARG, "null schedule");
  const bool fp32 = precision == LM_FP32_MIXED;
  for (const lm::Sched& c : sched_candidates(n, fp32, batched)) {
    if (c.tile == s->col_tile && c.remap == s->xcd_order && c.streams == s->streams) {
      put_sched(n, fp32, batched, c);
      return LM_OK;
    }
  }
  return fail(LM_E_ARG, "not a usable schedule for this n and precision");
}

lm_status get_schedule_ctx(int32_t n, int32_t precision, lm_schedule* s, bool batched) {
  if (!supported_n(n)) return fail(LM_E_UNSUPPORTED, "n must be 64, 128, 192, 256, 384, 512 or 1024");
  if (precision != LM_FP64 && precision != LM_FP32_MIXED) return fail(LM_E_ARG, "unknown precision");
  if (!s) return fail(LM_E_ARG, "null schedule");
  const lm::Sched c = get_sched(n, precision == LM_FP32_MIXED, batched);
  *s = lm_schedule{c.tile, c.remap, c.streams};
  return LM_OK;
}

}  // namespace

extern "C" {

lm_status lm_set_schedule(int32_t n, int32_t precision, const lm_schedule* s) {
  return set_schedule_ctx(n, precision, s, false);
}
lm_status lm_get_schedule(int32_t n, int32_t precision, lm_schedule* s) {
  return get_schedule_ctx(n, precision, s, false);
}
lm_status lm_set_batch_schedule(int32_t n, int32_t precision, const lm_schedule* s) {
  return set_schedule_ctx(n, precision, s, true);
}
lm_status lm_get_batch_schedule(int32_t n, int32_t precision, lm_schedule* s) {
  return get_schedule_ctx(n, precision, s, true);
}

lm_status lm_autotune(lm_run* r, int32_t steps, int32_t reps, lm_schedule* best, double* ms, int32_t cap,
                      int32_t* count) {
  if (!r) return fail(LM_E_ARG, "null run");
  if (r->batch) return fail(LM_E_STATE, "the run belongs to a batch");
  if (!r->has_state) return fail(LM_E_STATE, "no state set");
  if (steps < 1 || steps > 64) return fail(LM_E_ARG, "steps must be in 1..64");
  if (reps < 1 || reps > 16) return fail(LM_E_ARG, "reps must be in 1..16");
  if (cap < 0 || (cap > 0 && !ms)) return fail(LM_E_ARG, "cap < 0 or null ms");
  const std::vector<lm::Sched> cand = sched_candidates(r->d.N, r->fp32);
  const size_t bytes = r->L.total;
  void* snap = nullptr;
  if (hipMalloc(&snap, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LM_E_OOM, "autotune: no room for a copy of the run");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int64_t n0 = r->n, nt0 = r->n_tau;
  const int ys0 = r->ys_cur;
  const lm::Sched keep = r->sched;
  std::vector<double> best_ms(cand.size(), 0.0);
  // every exit below restores the run and frees the copy
  hipError_t e = hipMemcpyAsync(snap, r->slab, bytes, hipMemcpyDeviceToDevice, r->stream);
  const bool have_copy = (e == hipSuccess);
  auto restore = [&]() -> hipError_t {
    r->n = n0;
    r->n_tau = nt0;
    r->ys_cur = ys0;
    r->sched = keep;
    return have_copy ? hipMemcpyAsync(r->slab, snap, bytes, hipMemcpyDeviceToDevice, r->stream) : hipSuccess;
  };
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // one untimed step first: caches and clocks in their working state
  if (e == hipSuccess) {
    LM_DISPATCH_N(r->d.N, lm::launch_steps, *r, 1);
    e = hipGetLastError();
  }
  for (size_t k = 0; k < cand.size() && e == hipSuccess; ++k) {
    double bk = 0.0;
    for (int rep = 0; rep < reps && e == hipSuccess; ++rep) {
      e = restore();
      r->sched = cand[k];
      if (e == hipSuccess) e = hipEventRecord(e0, r->stream);
      if (e == hipSuccess) {
        LM_DISPATCH_N(r->d.N, lm::launch_steps, *r, steps);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipEventRecord(e1, r->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e == hipSuccess && (rep == 0 || t < bk)) bk = t;
    }
    best_ms[k] = bk / steps;
  }
  const hipError_t er = restore();
  const hipError_t es = hipStreamSynchronize(r->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(snap);
  if (e == hipSuccess) e = (er != hipSuccess) ? er : es;
  if (e != hipSuccess) return fail(LM_E_HIP, std::string("autotune: ") + hipGetErrorString(e));
  size_t bi = 0;
  for (size_t k = 1; k < cand.size(); ++k)
    if (best_ms[k] < best_ms[bi]) bi = k;
  put_sched(r->d.N, r->fp32, false, cand[bi]);
  if (best) *best = lm_schedule{cand[bi].tile, cand[bi].remap, cand[bi].streams};
  for (int k = 0; k < (int)cand.size() && k < cap; ++k) ms[k] = best_ms[k];
  if (count) *count = (int32_t)cand.size();
  return LM_OK;
}

lm_status lm_batch_destroy(lm_batch* b) {
  if (!b) return LM_OK;
  (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  for (auto& mm : b->members) mm.run->batch = nullptr;
  for (auto& g : b->groups) {
    if (g.d_desc) (void)hipFree(g.d_desc);
    if (g.fork) (void)hipStreamDestroy(g.fork);
    if (g.join) (void)hipEventDestroy(g.join);
  }
  if (b->d_counters) (void)hipFree(b->d_counters);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return LM_OK;
}

}  // extern "C"
