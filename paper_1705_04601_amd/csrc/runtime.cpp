// Runtime pieces shared by every entry point: errors, stream, device memory.
#include <algorithm>
#include <chrono>
#include <iterator>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "h2_internal.h"

namespace h2 {

static thread_local hipStream_t g_stream = nullptr;

hipStream_t current_stream() { return g_stream; }
void set_stream(hipStream_t s) { g_stream = s; }

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
int trace_level() {
  static const int lv = [] {
    const char* v = std::getenv("H2SP_TRACE");
    return v ? std::max(0, std::atoi(v)) : 0;
  }();
  return lv;
}
bool trace_enabled() { return trace_level() > 0; }
TraceTimer::TraceTimer(const char* n) : name(n), t0(now_ms()) {}
void TraceTimer::lap(const char* what) {
  const double t = now_ms();
  if (trace_enabled()) std::fprintf(stderr, "[h2sp] %s/%s %.1f ms\n", name, what, t - t0);
  t0 = t;
}
TraceTimer::~TraceTimer() {
  if (trace_enabled()) std::fprintf(stderr, "[h2sp] %s/end %.1f ms\n", name, now_ms() - t0);
}

void check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory) ? H2_ENOMEM : H2_EDEVICE;
  fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- device memory
// Caching allocator.  hipFree waits for the whole device, which serialises
// work queued on other streams (batched instances run on a stream pool), and
// the same large buffers come back call after call.  A freed block is kept
// with an event recorded on the freeing stream; a later request of about its
// size takes it back after making its own stream wait for that event.  Idle
// blocks are capped (the longest idle released first, so that the buffers of
// the work that runs now stay) and are all released when hipMalloc runs out.
namespace {
struct CachedBlock {
  void* p;
  size_t cap;
  hipEvent_t done;
  int dev;
  uint64_t seq;  // order of the frees
};
uint64_t g_seq = 0;
std::mutex g_cache_mu;
std::multimap<size_t, CachedBlock> g_cache;  // by capacity
size_t g_cached = 0;
// idle bytes kept: 90% of the device's memory by default
// (H2SP_DEVICE_CACHE_FRACTION), as a caching allocator that gives memory
// back only when an allocation fails.  A step of the largest workloads holds
// well over half of the memory (in FP64 at N = 1M: S 120 GB and the level
// buffers 80 GB), and a fresh hipMalloc maps pages at about 25 GB/s, so a
// smaller cache would map them again on every call.
size_t cache_limit() {
  static const size_t lim = [] {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || total_b == 0) {
      (void)hipGetLastError();
      return size_t(64) << 30;
    }
    double frac = 0.9;
    if (const char* e = std::getenv("H2SP_DEVICE_CACHE_FRACTION")) frac = std::min(1.0, std::max(0.0, std::atof(e)));
    return size_t(double(total_b) * frac);
  }();
  return lim;
}

size_t round_cap(size_t b) {
  constexpr size_t g = size_t(2) << 20;
  return b >= (size_t(1) << 20) ? (b + g - 1) & ~(g - 1) : (b + 255) & ~size_t(255);
}

// releases idle blocks (longest idle first) until at most `keep` bytes stay
// cached
void trim_locked(size_t keep) {
  while (g_cached > keep && !g_cache.empty()) {
    auto it = g_cache.begin();
    for (auto j = g_cache.begin(); j != g_cache.end(); ++j)
      if (j->second.seq < it->second.seq) it = j;
    (void)hipEventSynchronize(it->second.done);
    (void)hipEventDestroy(it->second.done);
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (it->second.dev != cur) (void)hipSetDevice(it->second.dev);
    (void)hipFree(it->second.p);
    if (it->second.dev != cur) (void)hipSetDevice(cur);
    g_cached -= it->second.cap;
    g_cache.erase(it);
  }
}

void* device_alloc(size_t bytes, size_t* cap, hipStream_t first_use) {
  const size_t want = round_cap(bytes);
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  {
    std::unique_lock<std::mutex> lk(g_cache_mu);
    // a cached block at most a quarter (+ 64 MiB) larger than the request
    const size_t limit = want + want / 4 + (size_t(64) << 20);
    for (auto it = g_cache.lower_bound(want); it != g_cache.end() && it->first <= limit; ++it) {
      if (it->second.dev != dev) continue;
      const CachedBlock c = it->second;
      g_cache.erase(it);
      g_cached -= c.cap;
      lk.unlock();
      const hipError_t e = hipStreamWaitEvent(first_use, c.done, 0);
      (void)hipEventDestroy(c.done);
      if (e != hipSuccess) {
        (void)hipDeviceSynchronize();  // cannot order the reuse: wait for everything instead
        (void)hipGetLastError();
      }
      *cap = c.cap;
      return c.p;
    }
  }
  void* p = nullptr;
  const double t0 = now_ms();
  hipError_t e = hipMalloc(&p, want);
  if (trace_enabled() && now_ms() - t0 > 20.0) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::fprintf(stderr, "[h2sp] hipMalloc %.2f GB took %.1f ms (cached idle %.2f GB in %zu blocks)\n", want / 1e9,
                 now_ms() - t0, g_cached / 1e9, g_cache.size());
  }
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      trim_locked(0);
    }
    e = hipMalloc(&p, want);
  }
  check_hip(e, "hipMalloc");
  *cap = want;
  return p;
}

void device_free(void* p, size_t cap) {
  int dev = 0;
  hipEvent_t ev = nullptr;
  if (hipGetDevice(&dev) != hipSuccess || hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, current_stream()) != hipSuccess) {
    if (ev) (void)hipEventDestroy(ev);
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    (void)hipFree(p);
    return;
  }
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.emplace(cap, CachedBlock{p, cap, ev, dev, ++g_seq});
  g_cached += cap;
  trim_locked(cache_limit());
}
}  // namespace

size_t cached_device_bytes() {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  return g_cached;
}

// ---------------------------------------------------------------- pinned pool
namespace {
std::mutex g_pin_mu;
std::multimap<size_t, char*> g_pin_free;  // idle blocks by capacity
size_t g_pin_idle = 0;
constexpr size_t kPinIdleLimit = size_t(8) << 30;  // idle pinned bytes kept
}  // namespace

PinnedBlock pinned_acquire(size_t bytes) {
  bytes = std::max<size_t>(bytes, 1);
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pin_free.lower_bound(bytes);
    if (it != g_pin_free.end() && it->first <= 2 * bytes + (size_t(64) << 20)) {
      PinnedBlock b{it->second, it->first};
      g_pin_idle -= it->first;
      g_pin_free.erase(it);
      return b;
    }
  }
  // a quarter more than asked, so that a slightly larger plan reuses it
  const size_t cap = ((bytes + bytes / 4) + 4095) & ~size_t(4095);
  void* p = nullptr;
  HIPCHECK(hipHostMalloc(&p, cap, hipHostMallocDefault));
  return PinnedBlock{static_cast<char*>(p), cap};
}

void pinned_release(PinnedBlock b) {
  if (!b.ptr) return;
  std::vector<char*> drop;
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.emplace(b.cap, b.ptr);
    g_pin_idle += b.cap;
    while (g_pin_idle > kPinIdleLimit && !g_pin_free.empty()) {  // largest first
      auto it = std::prev(g_pin_free.end());
      g_pin_idle -= it->first;
      drop.push_back(it->second);
      g_pin_free.erase(it);
    }
  }
  for (char* p : drop) (void)hipHostFree(p);
}

bool graphs_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("H2SP_GRAPHS");
    return !(v && v[0] == '0');
  }();
  return on;
}

LaunchGraph::~LaunchGraph() {
  if (exec) (void)hipGraphExecDestroy(exec);
}

void LaunchGraph::capture(const std::function<void(hipStream_t)>& record) {
  hipStream_t cap = nullptr;
  HIPCHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    record(cap);
    e = hipStreamEndCapture(cap, &graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) exec = nullptr;
  check_hip(e, "capturing a launch sequence");
}

DeviceBuffer::DeviceBuffer(size_t b) { reset(b); }

DeviceBuffer& DeviceBuffer::operator=(DeviceBuffer&& o) noexcept {
  if (this != &o) {
    if (ptr) device_free(ptr, cap);
    ptr = o.ptr;
    bytes = o.bytes;
    cap = o.cap;
    o.ptr = nullptr;
    o.bytes = 0;
    o.cap = 0;
  }
  return *this;
}

DeviceBuffer::~DeviceBuffer() {
  if (ptr) device_free(ptr, cap);
}

void DeviceBuffer::reset(size_t b, hipStream_t first_use) {
  if (ptr) {
    device_free(ptr, cap);
    ptr = nullptr;
    cap = 0;
  }
  bytes = b;
  if (b) ptr = device_alloc(b, &cap, first_use ? first_use : current_stream());
}

}  // namespace h2
