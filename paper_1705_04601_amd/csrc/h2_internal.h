// Internal data structures of libh2sp (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <parallel/algorithm>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/h2sp.h"

namespace h2 {

using i64 = int64_t;

// Error carried through the host code and turned into a status at the ABI.
struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define HIPCHECK(x) ::h2::check_hip((x), #x)

hipStream_t current_stream();

// Host-side phase timer: with H2SP_TRACE=1 in the environment each phase's
// wall time is printed to stderr as "[h2sp] <name> <ms> ms".
struct TraceTimer {
  const char* name;
  double t0;
  explicit TraceTimer(const char* n);
  void lap(const char* what);
  ~TraceTimer();
};
bool trace_enabled();  // H2SP_TRACE >= 1: phase timings and statistics on stderr
int trace_level();     // H2SP_TRACE >= 2 adds per-level lines

// ---------------------------------------------------------------- cluster tree
// Heap numbering: root 0, sons of c are 2c+1 and 2c+2; every leaf at depth L.
struct Tree {
  i64 n = 0;
  int dim = 0;
  int depth = 0;
  std::vector<i64> perm;       // tree position -> original index
  std::vector<i64> start;      // per cluster: first tree position
  std::vector<i64> size;       // per cluster: number of points
  std::vector<double> lo, hi;  // per cluster: tight box (ncl * dim)
  i64 ncl() const { return (i64(1) << (depth + 1)) - 1; }
  int level(i64 c) const;      // 0 = leaves
  i64 first_at_level(int k) const { return (i64(1) << (depth - k)) - 1; }
  i64 count_at_level(int k) const { return i64(1) << (depth - k); }
  bool is_leaf(i64 c) const { return 2 * c + 1 >= ncl(); }
};

struct Pair {
  int32_t t, s;
};

// Per level: near (inadmissible) and far (admissible) pairs, sorted by (t, s).
struct BlockTree {
  std::vector<std::vector<Pair>> near, far;
};

Tree build_tree(const double* pts, i64 n, int dim, int leaf);
BlockTree build_block_tree(const Tree& tr, double eta);
std::vector<char> farfield_flags(const Tree& tr, const BlockTree& bt);

// ---------------------------------------------------------------- device arena
// Device memory block from the library's caching allocator (a freed block is
// kept for reuse, ordered by an event on the freeing stream).
struct DeviceBuffer {
  void* ptr = nullptr;
  size_t bytes = 0;  // requested
  size_t cap = 0;    // allocated
  DeviceBuffer() = default;
  explicit DeviceBuffer(size_t b);
  DeviceBuffer(const DeviceBuffer&) = delete;
  DeviceBuffer& operator=(const DeviceBuffer&) = delete;
  DeviceBuffer(DeviceBuffer&& o) noexcept : ptr(o.ptr), bytes(o.bytes), cap(o.cap) {
    o.ptr = nullptr;
    o.bytes = 0;
    o.cap = 0;
  }
  DeviceBuffer& operator=(DeviceBuffer&& o) noexcept;
  ~DeviceBuffer();
  // frees the block (ordered after the work queued on the current stream) and
  // allocates b bytes; a reused block is made safe for `first_use` (default:
  // the current stream), the stream that touches it first
  void reset(size_t b, hipStream_t first_use = nullptr);
  template <class T> T* as() const { return static_cast<T*>(ptr); }
};

// Sort of a random-access range: in parallel (GNU parallel mode, OpenMP) when
// it is long, plainly when it is short (the parallel sort's team start costs
// more than a short sort, and plans run many of them, one per level).
template <class It>
void sort_range(It first, It last) {
  if (last - first >= (1 << 17)) __gnu_parallel::sort(first, last);
  else std::sort(first, last);
}

// Bytes held by idle cached blocks (free for the library's own allocations).
size_t cached_device_bytes();

// Page-locked host staging memory for uploads (hipHostMalloc), kept in a pool
// for reuse: a copy from it runs at the link's speed and without the
// runtime's own staging.  The block is the caller's until released.
struct PinnedBlock {
  char* ptr = nullptr;
  size_t cap = 0;
};
PinnedBlock pinned_acquire(size_t bytes);
void pinned_release(PinnedBlock b);

// A fixed sequence of kernel launches (a plan's sweep) captured once into a
// HIP graph on a private stream and replayed on the caller's stream; the
// sequence must only launch kernels.  H2SP_GRAPHS=0 runs it eagerly instead.
bool graphs_enabled();
struct LaunchGraph {
  hipGraphExec_t exec = nullptr;
  LaunchGraph() = default;
  LaunchGraph(const LaunchGraph&) = delete;
  LaunchGraph& operator=(const LaunchGraph&) = delete;
  ~LaunchGraph();
  void capture(const std::function<void(hipStream_t)>& record);
  template <class F>
  void run(hipStream_t st, F&& record) {
    if (!graphs_enabled()) {
      record(st);
      return;
    }
    if (!exec) capture(record);
    HIPCHECK(hipGraphLaunch(exec, st));
  }
};

template <class T>
DeviceBuffer upload(const std::vector<T>& v) {
  DeviceBuffer d(v.size() * sizeof(T));
  if (!v.empty())
    HIPCHECK(hipMemcpyAsync(d.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice,
                            current_stream()));
  return d;
}

}  // namespace h2

// ---------------------------------------------------------------- H^2 matrix
struct h2_matrix {
  h2::Tree tree;
  h2::BlockTree bt;
  std::vector<char> ff;           // cluster carries a basis
  std::vector<double> x_tree;     // points in tree order (n * dim)
  double scale = 0, diag = 0;
  int kern = H2_KERNEL_INVDIST;   // h2_kernel::kind
  double kparam = 0;              // h2_kernel::param (d of H2_KERNEL_IFMM)
  int cheb = 0, P = 0;            // nodes per axis, nodes per cluster
  bool identity_proj = false;     // P_t = I (no recompression)
  std::vector<int32_t> rank;      // r_t
  std::vector<double> nodes;      // ncl * P * dim (row-major per cluster)
  std::vector<h2::i64> proj_off;  // offset of P_t (r_t x P col-major) or -1
  std::vector<double> proj;
  std::vector<h2::i64> basis_off; // leaves: offset of R_t (|t| x r_t col-major) or -1
  std::vector<double> basis;
  std::vector<h2::i64> transfer_off;  // offset of T_c (r_c x r_father col-major) or -1
  std::vector<double> transfer;
  // device copies
  h2::DeviceBuffer d_x, d_nodes, d_proj, d_basis, d_transfer, d_perm;
  bool on_device = false;
  void upload_all();   // copies the coefficients to the current device (once)
};
