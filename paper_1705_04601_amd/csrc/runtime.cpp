// Runtime pieces shared by every entry point: errors, stream, device memory.
#include <chrono>
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
bool trace_enabled() {
  static const bool on = [] {
    const char* v = std::getenv("H2SP_TRACE");
    return v && v[0] && v[0] != '0';
  }();
  return on;
}
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

DeviceBuffer::DeviceBuffer(size_t b) { reset(b); }

DeviceBuffer& DeviceBuffer::operator=(DeviceBuffer&& o) noexcept {
  if (this != &o) {
    if (ptr) (void)hipFree(ptr);
    ptr = o.ptr;
    bytes = o.bytes;
    o.ptr = nullptr;
    o.bytes = 0;
  }
  return *this;
}

DeviceBuffer::~DeviceBuffer() {
  if (ptr) (void)hipFree(ptr);
}

void DeviceBuffer::reset(size_t b) {
  if (ptr) {
    HIPCHECK(hipStreamSynchronize(current_stream()));
    HIPCHECK(hipFree(ptr));
    ptr = nullptr;
  }
  bytes = b;
  if (b) HIPCHECK(hipMalloc(&ptr, b));
}

}  // namespace h2
