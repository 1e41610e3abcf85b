// Host-only model of the HIP runtime and of the solver entry points the
// serving pool calls, so that the pool's bookkeeping (arena, slots, graph
// capture and retirement, harvesting) can run on the CPU under
// AddressSanitizer.  The "device" is one FIFO of deferred operations that the
// driver advances at random points (mock_progress); device memory is host
// memory.  Each job workspace carries a tag naming the job that owns it, and
// every deferred operation of a job checks that tag, so work that runs after
// its workspace was handed to another job is reported.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <vector>

#include "lfsr_handle.h"

struct MockStream { int id; };
struct MockEvent { uint64_t recorded = 0, completed = 0; };
struct MockGraph { std::vector<std::function<void()>> nodes; };
struct MockExec { std::vector<std::function<void()>> nodes; };

namespace {
std::deque<std::function<void()>> g_queue;
MockGraph* g_cap = nullptr;
hipStream_t g_cap_stream = nullptr;
std::map<const lfsr_handle*, uint64_t> g_serial;
uint64_t g_next_serial = 1;

struct WsTag { uint64_t serial; int64_t iters; };
constexpr size_t kTagAt = 256;

[[noreturn]] void fail(const char* what) {
  std::fprintf(stderr, "mock runtime: %s\n", what);
  std::abort();
}

void enqueue(std::function<void()> f) {
  if (g_cap) g_cap->nodes.push_back(std::move(f));
  else g_queue.push_back(std::move(f));
}

void run_one() {
  std::function<void()> f = std::move(g_queue.front());
  g_queue.pop_front();
  f();
}

void check_tag(char* ws, uint64_t serial) {
  if (reinterpret_cast<WsTag*>(ws + kTagAt)->serial != serial) fail("job work ran on a workspace owned by another job");
}
}  // namespace

// Error injection: the n-th later call of hipMemcpyAsync / hipEventQuery
// fails (n < 0: never).
long g_memcpy_fail = -1, g_query_fail = -1;
extern "C" void mock_fail_memcpy_in(long n) { g_memcpy_fail = n; }
extern "C" void mock_fail_query_in(long n) { g_query_fail = n; }

extern "C" void mock_progress(size_t n) {
  while (n-- > 0 && !g_queue.empty()) run_one();
}
extern "C" size_t mock_pending() { return g_queue.size(); }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  static int id = 0;
  *s = new MockStream{++id};
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (s == g_cap_stream) fail("stream destroyed while capturing");
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) {
  if (g_cap) fail("synchronize while capturing");
  while (!g_queue.empty()) run_one();
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) {
  if (!e) return hipErrorInvalidValue;
  return hipSuccess;  // one FIFO: every wait is already satisfied by order
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new MockEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;  // a pending record of it then touches freed memory (reported by the sanitizer)
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  if (!e) return hipErrorInvalidValue;
  if (g_cap) return hipSuccess;  // inside a capture an event only orders the captured work
  const uint64_t n = ++e->recorded;
  g_queue.push_back([e, n] { e->completed = n; });
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  if (g_query_fail >= 0 && g_query_fail-- == 0) return hipErrorInvalidValue;
  return e->completed == e->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (g_cap) fail("event synchronize while capturing");
  while (e->completed != e->recorded) {
    if (g_queue.empty()) fail("event can never complete");
    run_one();
  }
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  *p = std::calloc(1, bytes);
  return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  if (g_memcpy_fail >= 0 && g_memcpy_fail-- == 0) return hipErrorInvalidValue;
  enqueue([dst, src, bytes] { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (g_cap) fail("nested capture");
  g_cap = new MockGraph();
  g_cap_stream = s;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!g_cap || s != g_cap_stream) fail("end of a capture that was not begun on this stream");
  *g = g_cap;
  g_cap = nullptr;
  g_cap_stream = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *x = new MockExec{g->nodes};
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;  // a pending launch of it then touches freed memory (reported by the sanitizer)
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) {
  if (g_cap) fail("graph launch while capturing");
  g_queue.push_back([x] {
    for (auto& f : x->nodes) f();
  });
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "mock error"; }

// Solver entry points: a job's "state" is its tag and its DevScalars.
size_t lfsr_workspace_bytes(const lfsr_params* p) {
  if (!p || p->lr_h < 1 || p->lr_w < 1 || p->admm_iters < 1) return 0;
  return 512 + (size_t)p->lr_h * p->lr_w * 64;
}
lfsr_status lfsr_create(const lfsr_params* p, void* ws, size_t bytes, lfsr_handle** out) {
  const size_t need = lfsr_workspace_bytes(p);
  if (!need || !ws || bytes < need || !out) return LFSR_ENOMEM;
  lfsr_handle* h = new lfsr_handle();
  h->prm = *p;
  h->ws = static_cast<char*>(ws);
  h->b.sc = reinterpret_cast<lfsr::DevScalars*>(ws);
  h->n_done = 0;
  h->bound = false;
  h->broken = false;
  g_serial[h] = g_next_serial++;
  *out = h;
  return LFSR_OK;
}
void lfsr_destroy(lfsr_handle* h) {
  if (!h) return;
  g_serial.erase(h);
  delete h;
}
const char* lfsr_last_error(const lfsr_handle* h) { return h ? h->err.c_str() : "mock"; }
lfsr_status lfsr_init(lfsr_handle* h, const float* d_lr, const float* d_disp, const float*, const float*, void*) {
  if (!d_lr || !d_disp) return LFSR_EINVAL;
  char* ws = h->ws;
  const uint64_t serial = g_serial.at(h);
  h->y = d_lr;
  enqueue([ws, serial] {
    std::memset(ws, 0, sizeof(lfsr::DevScalars));
    *reinterpret_cast<WsTag*>(ws + kTagAt) = WsTag{serial, 0};
  });
  h->bound = true;
  return LFSR_OK;
}
lfsr_status lfsr_iterate(lfsr_handle* h, int32_t count, void*) {
  if (!h->bound) return LFSR_ESTATE;
  char* ws = h->ws;
  const uint64_t serial = g_serial.at(h);
  const float* y = h->y;
  for (int i = 0; i < count; ++i) {
    enqueue([ws, serial, y] {
      check_tag(ws, serial);
      volatile float v = y[0];  // the job's inputs must still be alive
      (void)v;
      reinterpret_cast<WsTag*>(ws + kTagAt)->iters += 1;
      reinterpret_cast<lfsr::DevScalars*>(ws)->iters_done += 1;
    });
  }
  h->n_done += count;
  return LFSR_OK;
}
lfsr_status lfsr_read_state(lfsr_handle* h, float* d_x, float*, float*, float*, void*) {
  char* ws = h->ws;
  const uint64_t serial = g_serial.at(h);
  enqueue([ws, serial, d_x] {
    check_tag(ws, serial);
    if (d_x) d_x[0] = (float)reinterpret_cast<WsTag*>(ws + kTagAt)->iters;
  });
  return LFSR_OK;
}
