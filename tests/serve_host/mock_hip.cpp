// Host-only model of the HIP runtime under the library's real host code
// (lfsr_api, lfsr_pool and the kernel launchers of lfsr_kernels, compiled for
// the host side only), so that the solver's planning, launch and serving-pool
// paths run on the CPU under AddressSanitizer and UBSan.
//
// Kernels are registered through the compiler's registration calls and every
// launch is checked (registered kernel, live stream, grid and block limits,
// dynamic LDS within the 160 KiB of a CU) and recorded, not run.  The device
// is one FIFO of deferred operations that the driver advances at random points
// (mock_progress); copies touch the first and last byte of both buffers, so a
// copy that runs after its host or device buffer was freed is reported by the
// sanitizer.  Stream capture follows HIP's rules for the calls the library
// makes: a stream joins a capture by waiting on an event recorded inside it,
// every joined stream must be joined back before the capture ends, and
// synchronising calls during a capture are errors.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <set>
#include <string>
#include <vector>

struct ihipStream_t {
  int id;
  bool capturing = false;      // part of the running capture
  bool origin = false;         // the stream the capture began on
  bool joined_back = true;     // its last captured work is joined to the origin
};
struct ihipEvent_t {
  unsigned long recorded = 0, completed = 0;
  ihipStream_t* captured_on = nullptr;  // recorded inside the running capture, on this stream
  bool captured = false;
};
struct ihipGraph {
  std::vector<std::function<void()>> nodes;
};
struct hipGraphExec {
  std::vector<std::function<void()>> nodes;
};

namespace {

struct Kernel {
  std::string name;
  size_t max_lds = 0;
  long launches = 0;
};

std::deque<std::function<void()>> g_queue;
ihipGraph* g_cap = nullptr;
std::set<ihipStream_t*> g_streams;  // live streams
std::vector<ihipStream_t*> g_cap_streams;
// function-local: registration runs from other objects' constructors
std::map<const void*, Kernel>& kernels() {
  static std::map<const void*, Kernel> k;
  return k;
}
hipError_t g_last = hipSuccess;
struct Config {
  dim3 grid, block;
  size_t shmem;
  hipStream_t stream;
};
std::vector<Config> g_config;
long g_launches = 0, g_graph_nodes_max = 0;

[[noreturn]] void fail(const std::string& what) {
  std::fprintf(stderr, "mock hip: %s\n", what.c_str());
  std::fflush(stderr);
  std::abort();
}

void check_stream(hipStream_t s, const char* where) {
  if (s && !g_streams.count(s)) fail(std::string(where) + ": stream not alive");
}

bool in_capture(hipStream_t s) { return g_cap && s && s->capturing; }

void enqueue(hipStream_t s, std::function<void()> f) {
  if (g_cap && s == nullptr) fail("work on the null stream during a capture");
  if (in_capture(s)) {
    s->joined_back = false;
    g_cap->nodes.push_back(std::move(f));
  } else {
    g_queue.push_back(std::move(f));
  }
}

void run_one() {
  std::function<void()> f = std::move(g_queue.front());
  g_queue.pop_front();
  f();
}

void drain() {
  while (!g_queue.empty()) run_one();
}

void touch(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  volatile const char* s = static_cast<const char*>(src);
  volatile char* d = static_cast<char*>(dst);
  const char a = s[0], b = s[bytes - 1];
  d[0] = a;
  d[bytes - 1] = b;
}

}  // namespace

// -- driver hooks
extern "C" void mock_progress(size_t n) {
  while (n-- > 0 && !g_queue.empty()) run_one();
}
extern "C" size_t mock_pending() { return g_queue.size(); }
extern "C" void mock_report() {
  std::printf("mock hip: %ld kernel launches recorded, largest graph %ld nodes, %zu kernels used\n", g_launches,
              g_graph_nodes_max, kernels().size());
  size_t lds = 0;
  for (auto& kv : kernels()) lds = kv.second.max_lds > lds ? kv.second.max_lds : lds;
  std::printf("mock hip: largest dynamic LDS of a launch %zu bytes\n", lds);
}

// -- compiler registration calls
extern "C" void** __hipRegisterFatBinary(void* wrapper) {
  static void* modules[1];
  (void)wrapper;
  return modules;
}
extern "C" void __hipUnregisterFatBinary(void**) {}
extern "C" void __hipRegisterFunction(void**, const void* host_fn, char*, const char* device_name, unsigned int,
                                      void*, void*, dim3*, dim3*, int*) {
  kernels()[host_fn].name = device_name;
}
extern "C" void __hipRegisterVar(void**, void*, char*, char*, int, size_t, int, int) {}

hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream) {
  g_config.push_back(Config{grid, block, shmem, stream});
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shmem, hipStream_t* stream) {
  if (g_config.empty()) fail("pop of a launch configuration that was not pushed");
  const Config c = g_config.back();
  g_config.pop_back();
  *grid = c.grid;
  *block = c.block;
  *shmem = c.shmem;
  *stream = c.stream;
  return hipSuccess;
}
hipError_t hipLaunchKernel(const void* fn, dim3 grid, dim3 block, void** args, size_t shmem, hipStream_t s) {
  auto it = kernels().find(fn);
  if (it == kernels().end()) fail("launch of an unregistered kernel");
  check_stream(s, "hipLaunchKernel");
  if (!args) fail("launch without an argument array");
  const unsigned long long threads = (unsigned long long)block.x * block.y * block.z;
  if (grid.x == 0 || grid.y == 0 || grid.z == 0 || grid.x > 0x7fffffffu || grid.y > 65535 || grid.z > 65535 ||
      threads == 0 || threads > 1024 || shmem > 160 * 1024) {
    std::fprintf(stderr, "mock hip: bad launch of %s: grid (%u,%u,%u) block (%u,%u,%u) lds %zu\n",
                 it->second.name.c_str(), grid.x, grid.y, grid.z, block.x, block.y, block.z, shmem);
    g_last = hipErrorInvalidConfiguration;
    return g_last;
  }
  if (shmem > it->second.max_lds) it->second.max_lds = shmem;
  it->second.launches += 1;
  g_launches += 1;
  enqueue(s, [] {});
  return hipSuccess;
}
hipError_t hipGetLastError(void) {
  const hipError_t e = g_last;
  g_last = hipSuccess;
  return e;
}
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "mock error"; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  *p = const_cast<void*>(symbol);  // host memory stands for device memory here
  return hipSuccess;
}

// -- streams and events
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  static int id = 0;
  *s = new ihipStream_t{++id};
  g_streams.insert(*s);
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  check_stream(s, "hipStreamDestroy");
  if (s->capturing) fail("stream destroyed while capturing");
  g_streams.erase(s);
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  check_stream(s, "hipStreamSynchronize");
  if (g_cap) fail("synchronize during a capture");
  drain();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new ihipEvent_t();
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;  // a pending record of it then touches freed memory (reported by the sanitizer)
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (!e) return hipErrorInvalidValue;
  check_stream(s, "hipEventRecord");
  if (in_capture(s)) {  // inside a capture an event only orders the captured work
    e->captured = true;
    e->captured_on = s;
    return hipSuccess;
  }
  if (g_cap && s == nullptr) fail("event record on the null stream during a capture");
  e->captured = false;
  const unsigned long n = ++e->recorded;
  g_queue.push_back([e, n] { e->completed = n; });
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  if (!e) return hipErrorInvalidValue;
  check_stream(s, "hipStreamWaitEvent");
  if (e->captured && g_cap) {
    if (!s) fail("null stream joins a capture");
    if (!s->capturing) {  // the stream joins the capture
      s->capturing = true;
      s->joined_back = true;
      g_cap_streams.push_back(s);
    }
    if (s->origin && e->captured_on) e->captured_on->joined_back = true;
    return hipSuccess;
  }
  return hipSuccess;  // one FIFO: every wait is satisfied by order
}
hipError_t hipEventQuery(hipEvent_t e) { return e->completed == e->recorded ? hipSuccess : hipErrorNotReady; }
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (g_cap) fail("event synchronize during a capture");
  while (e->completed != e->recorded) {
    if (g_queue.empty()) fail("event can never complete");
    run_one();
  }
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}

// -- memory
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
  *p = std::calloc(1, bytes);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  check_stream(s, "hipMemcpyAsync");
  if (!dst || !src) return hipErrorInvalidValue;
  if (bytes <= 4096)
    enqueue(s, [dst, src, bytes] { std::memcpy(dst, src, bytes); });
  else
    enqueue(s, [dst, src, bytes] { touch(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  if (g_cap) fail("synchronous copy during a capture");
  drain();
  if (bytes <= 4096) std::memcpy(dst, src, bytes);
  else touch(dst, src, bytes);
  return hipSuccess;
}

// -- graphs
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  check_stream(s, "hipStreamBeginCapture");
  if (!s) fail("capture on the null stream");
  if (g_cap) fail("nested capture");
  g_cap = new ihipGraph();
  s->capturing = true;
  s->origin = true;
  s->joined_back = true;
  g_cap_streams.assign(1, s);
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!g_cap || !s || !s->origin) fail("end of a capture that was not begun on this stream");
  for (ihipStream_t* b : g_cap_streams) {
    if (b != s && !b->joined_back) fail("capture ended with a branch that was not joined back");
    b->capturing = false;
    b->origin = false;
  }
  g_cap_streams.clear();
  if ((long)g_cap->nodes.size() > g_graph_nodes_max) g_graph_nodes_max = (long)g_cap->nodes.size();
  *g = g_cap;
  g_cap = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *x = new hipGraphExec{g->nodes};
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
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  check_stream(s, "hipGraphLaunch");
  if (g_cap) fail("graph launch during a capture");
  g_queue.push_back([x] {
    for (auto& f : x->nodes) f();
  });
  return hipSuccess;
}
