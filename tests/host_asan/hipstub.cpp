// A stand-in for the HIP runtime, for host-only sanitizer runs of the C ABI on
// a machine without a GPU.  Test infrastructure only.
//
// "Device" memory is host memory (so AddressSanitizer sees every copy into and
// out of it).  Kernels do nothing; their launch shapes are checked.  Work on a
// stream is deferred, as on a GPU: asynchronous copies, fills and kernels are
// queued and only carried out when something waits for that stream (a stream
// or event synchronisation, a blocking copy, hipFree).  So an asynchronous copy
// into a caller's buffer or a stack variable that outlives the call that issued
// it is carried out late, and the sanitizer reports the stale access.  Stream
// capture records the queued operations of every stream that joins the capture
// into a graph; launching the instantiated graph queues them again.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

namespace {

using Op = std::function<void()>;

struct Graph {
  std::vector<Op> ops;
};

struct Stream {
  std::deque<Op> queue;
  Graph* capture = nullptr;  // graph being captured into, if any
  Stream* origin = nullptr;  // the stream the capture began on
};

struct Event {
  Stream* stream = nullptr;  // stream of the last record
};

std::recursive_mutex g_mu;
Stream g_null;  // stream 0
std::vector<std::unique_ptr<Stream>> g_streams;
std::map<void*, size_t> g_allocs;  // live device allocations
hipError_t g_last = hipSuccess;

struct Var {
  size_t size;
  void* dev = nullptr;
};
std::map<const void*, Var> g_vars;  // registered device variables, by host shadow

[[noreturn]] void die(const char* what) {
  std::fprintf(stderr, "hipstub: %s\n", what);
  std::fflush(stderr);
  std::abort();
}

Stream* S(hipStream_t s) {
  if (!s) return &g_null;
  for (auto& p : g_streams)
    if ((hipStream_t)p.get() == s) return p.get();
  die("unknown stream handle");
}

void flush(Stream* s) {
  if (s->capture) die("synchronising a stream during capture");
  while (!s->queue.empty()) {
    Op op = std::move(s->queue.front());
    s->queue.pop_front();
    op();
  }
}

void flush_all() {
  flush(&g_null);
  for (auto& p : g_streams)
    if (!p->capture) flush(p.get());
}

void submit(Stream* s, Op op) {
  if (s->capture) s->capture->ops.push_back(std::move(op));
  else s->queue.push_back(std::move(op));
}

// a device range must lie inside one live allocation (or a registered variable)
void check_dev(const void* p, size_t n, const char* what) {
  if (n == 0) return;
  const char* c = (const char*)p;
  for (auto& v : g_vars)
    if (v.second.dev && c >= (const char*)v.second.dev && c + n <= (const char*)v.second.dev + v.second.size) return;
  auto it = g_allocs.upper_bound((void*)c);
  if (it != g_allocs.begin()) {
    --it;
    const char* b = (const char*)it->first;
    if (c >= b && c + n <= b + it->second) return;
  }
  std::fprintf(stderr, "hipstub: %s: %zu bytes at %p are not inside one device allocation\n", what, n, p);
  die("device range check failed");
}

bool is_device(const void* p) {
  auto it = g_allocs.upper_bound((void*)p);
  if (it != g_allocs.begin()) {
    --it;
    if ((const char*)p < (const char*)it->first + it->second) return true;
  }
  for (auto& v : g_vars)
    if (v.second.dev && p >= v.second.dev && (const char*)p < (const char*)v.second.dev + v.second.size) return true;
  return false;
}

void copy_checked(void* dst, const void* src, size_t n, hipMemcpyKind kind) {
  switch (kind) {
    case hipMemcpyHostToDevice: check_dev(dst, n, "copy to device"); break;
    case hipMemcpyDeviceToHost: check_dev(src, n, "copy from device"); break;
    case hipMemcpyDeviceToDevice:
      check_dev(dst, n, "device copy destination");
      check_dev(src, n, "device copy source");
      break;
    default: break;
  }
  std::memmove(dst, src, n);
}

struct Config {
  dim3 grid, block;
  size_t shm;
  hipStream_t stream;
};
thread_local std::vector<Config> t_cfg;

}  // namespace

extern "C" {

void** __hipRegisterFatBinary(const void*) {
  static void* handle[4] = {};
  return handle;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, uint3*, uint3*, dim3*, dim3*,
                           int*) {}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_vars[var] = Var{size, nullptr};
}

}  // extern "C"

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shm, hipStream_t stream) {
  t_cfg.push_back(Config{grid, block, shm, stream});
  return hipSuccess;
}

hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shm, hipStream_t* stream) {
  if (t_cfg.empty()) die("pop without push");
  const Config c = t_cfg.back();
  t_cfg.pop_back();
  *grid = c.grid;
  *block = c.block;
  *shm = c.shm;
  *stream = c.stream;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void*, dim3 grid, dim3 block, void**, size_t, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  const unsigned long long threads = 1ull * block.x * block.y * block.z;
  if (threads == 0 || threads > 1024 || grid.x == 0 || grid.y == 0 || grid.z == 0 || grid.y > 65535 ||
      grid.z > 65535) {
    std::fprintf(stderr, "hipstub: bad launch grid (%u,%u,%u) block (%u,%u,%u)\n", grid.x, grid.y, grid.z, block.x,
                 block.y, block.z);
    g_last = hipErrorInvalidConfiguration;
    return g_last;
  }
  submit(S(stream), [] {});
  return hipSuccess;
}

hipError_t hipGetLastError() {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}

const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "hipstub error"; }

hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}

hipError_t hipRuntimeGetVersion(int* v) {
  *v = HIP_VERSION;
  return hipSuccess;
}

hipError_t hipMalloc(void** p, size_t n) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!p) return hipErrorInvalidValue;
  void* q = std::aligned_alloc(256, (n + 255) / 256 * 256 + 256);
  if (!q) return hipErrorOutOfMemory;
  g_allocs[q] = n;
  *p = q;
  return hipSuccess;
}

hipError_t hipFree(void* p) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  if (!p) return hipSuccess;
  flush_all();  // hipFree waits for the device
  auto it = g_allocs.find(p);
  if (it == g_allocs.end()) die("hipFree of a pointer that is not a live allocation");
  g_allocs.erase(it);
  std::free(p);
  return hipSuccess;
}

hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  auto it = g_vars.find(symbol);
  if (it == g_vars.end()) return hipErrorInvalidSymbol;
  if (!it->second.dev) it->second.dev = std::calloc(1, it->second.size);
  *p = it->second.dev;
  return hipSuccess;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind kind) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  flush_all();
  copy_checked(dst, src, n, kind);
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  submit(S(stream), [=] { copy_checked(dst, src, n, kind); });
  return hipSuccess;
}

hipError_t hipMemset(void* dst, int v, size_t n) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  flush_all();
  check_dev(dst, n, "memset");
  std::memset(dst, v, n);
  return hipSuccess;
}

hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  Stream* s = S(stream);
  if (s->capture) die("hipMemsetAsync recorded into a captured graph");
  submit(s, [=] {
    check_dev(dst, n, "memset");
    std::memset(dst, v, n);
  });
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  g_streams.push_back(std::make_unique<Stream>());
  *s = (hipStream_t)g_streams.back().get();
  return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  Stream* p = S(s);
  if (p == &g_null) die("destroying the null stream");
  flush(p);
  for (auto it = g_streams.begin(); it != g_streams.end(); ++it)
    if (it->get() == p) {
      g_streams.erase(it);
      break;
    }
  return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  flush(S(s));
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  *e = (hipEvent_t) new Event();
  return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int) { return hipEventCreate(e); }

hipError_t hipEventDestroy(hipEvent_t e) {
  delete (Event*)e;
  return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  Event* ev = (Event*)e;
  Stream* st = S(s);
  ev->stream = st;
  submit(st, [] {});
  return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  Event* ev = (Event*)e;
  if (ev->stream) flush(ev->stream);
  return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.0f;
  return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  Event* ev = (Event*)e;
  Stream* st = S(s);
  if (ev->stream && ev->stream->capture && !st->capture) {
    // a stream that waits on a captured event joins the capture
    if (!st->queue.empty()) die("a stream with pending work joins a capture");
    st->capture = ev->stream->capture;
    st->origin = ev->stream->origin;
  } else if (ev->stream && !ev->stream->capture && ev->stream != st) {
    flush(ev->stream);  // stream order: the waited-for work happens first
  }
  return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  Stream* st = S(s);
  if (st->capture) die("capture begun twice");
  if (!st->queue.empty()) flush(st);
  st->capture = new Graph();
  st->origin = st;
  return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  Stream* st = S(s);
  if (!st->capture || st->origin != st) die("end of a capture that was not begun on this stream");
  Graph* graph = st->capture;
  for (auto& p : g_streams)
    if (p->capture == graph) {
      p->capture = nullptr;
      p->origin = nullptr;
    }
  if (g_null.capture == graph) g_null.capture = nullptr;
  *g = (hipGraph_t)graph;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *exec = (hipGraphExec_t) new Graph(*(Graph*)g);
  return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s) {
  std::lock_guard<std::recursive_mutex> lk(g_mu);
  Stream* st = S(s);
  for (const Op& op : ((Graph*)exec)->ops) submit(st, op);
  return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
  delete (Graph*)exec;
  return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g) {
  delete (Graph*)g;
  return hipSuccess;
}
