// Host-side builder of batched GEMM launches (items, K-segments, tile list).
#pragma once

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "h2_internal.h"
#include "kernels.h"
#include "tune.h"

namespace h2 {

// Allocator that leaves trivially constructible elements uninitialised on
// resize (work lists are written in full right after they are sized).
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
template <class T>
using PodVector = std::vector<T, NoInitAlloc<T>>;

// Work list of one batched GEMM launch.  Built on the host, copied to the
// device by upload_batches (one allocation for a whole plan), replayed as often
// as the plan is run.
struct GemmBatch {
  std::vector<GemmItem> items;
  std::vector<GemmSeg> segs;
  std::vector<int32_t> tiles;
  const GemmItem* d_items = nullptr;
  const GemmSeg* d_segs = nullptr;
  const int32_t* d_tiles = nullptr;
  int32_t ntiles = 0;
  int mode = GEMM_STORE;
  int role = ROLE_TRANSFORM;
  int amode = -1, bmode = -1;  // operand layouts shared by every segment (build_tiles)
  int kern = 0;                // kernel of generated operands, one per launch (build_tiles)
  int prec = -1;               // 0 FP64, 1 FP32: set by the planner, selects the tile table
  int variant = 0;             // output tile shape (gemm_shape), from the tuning table
  int wg_rows = 1;             // row tiles per work-group (build_tiles)
  double flops = 0.0;  // algorithmic flops of the batch

  bool empty() const { return items.empty(); }

  // Opens an item with output M x N; segments follow until the next item.
  GemmItem& item(int M, int N, int rs, int cs) {
    if (M > 512 || N > 512) fail(H2_EUNSUPPORTED, "GEMM item larger than 512 x 512");
    GemmItem it{};
    it.M = M;
    it.N = N;
    it.rs = rs;
    it.cs = cs;
    it.seg_begin = it.seg_end = int32_t(segs.size());
    items.push_back(it);
    return items.back();
  }
  static void set_out(GemmItem& it, int q, void* p, int64_t ld, bool trans) {
    it.out[q] = p;
    it.ld[q] = int32_t(ld);
    it.trans[q] = trans ? 1 : 0;
  }
  // A (M x K) times B (K x N) added to the open item.
  void seg(const void* A, int lda, bool tA, const void* B, int ldb, bool tB, int K) {
    GemmSeg s{};
    s.A = A;
    s.B = B;
    s.pc = nullptr;
    s.K = K;
    s.lda = lda;
    s.ldb = ldb;
    s.opA = tA;
    s.opB = tB;
    s.gen = 0;
    s.diag = 0;
    push(s);
  }
  // Generated B(k, j) = scale / |pr_j - pc_k| (diagonal value where j == k if
  // diag) times a stored A (M x K).
  void seg_genB(const void* A, int lda, bool tA, const double* pr, const double* pc, bool diag, int K) {
    GemmSeg s{};
    s.A = A;
    s.B = pr;
    s.pc = pc;
    s.K = K;
    s.lda = lda;
    s.ldb = 0;
    s.opA = tA;
    s.opB = 0;
    s.gen = 2;
    s.diag = diag ? 1 : 0;
    push(s);
  }
  // Generated A(i, k) = scale / |pr_i - pc_k| (diagonal value where i == k if diag).
  void seg_gen(const double* pr, const double* pc, bool diag, const void* B, int ldb, bool tB, int K) {
    GemmSeg s{};
    s.A = pr;
    s.B = B;
    s.pc = pc;
    s.K = K;
    s.lda = 0;
    s.ldb = ldb;
    s.opA = 0;
    s.opB = tB;
    s.gen = 1;
    s.diag = diag ? 1 : 0;
    push(s);
  }
  void push(const GemmSeg& s) {
    if (s.K <= 0) return;
    segs.push_back(s);
    GemmItem& it = items.back();
    it.seg_end = int32_t(segs.size());
    flops += 2.0 * it.M * double(it.N) * s.K;
  }
  // Tile list: one tile per work-group.  Items without segments are kept
  // only when they store (they then write zeros).
  void build_tiles() {
    tiles.clear();
    amode = bmode = -1;
    for (const GemmSeg& sg : segs) {
      const int am = sg.gen == 1 ? 2 : (sg.opA ? 0 : 1);
      const int bm = sg.gen == 2 ? 2 : (sg.opB ? 1 : 0);
      if (amode < 0) {
        amode = am;
        bmode = bm;
      } else if (am != amode || bm != bmode) {
        fail(H2_EINVAL, "internal: segments of one GEMM batch with different operand layouts");
      }
    }
    if (amode >= 0 && !gemm_layout_supported(role, amode, bmode))
      fail(H2_EINVAL, "internal: no GEMM kernel for this role and operand layout");
    kern = items.empty() ? 0 : items[0].gkern;
    if (amode == 2 || bmode == 2)
      for (const GemmItem& it : items)
        if (it.gkern != kern) fail(H2_EUNSUPPORTED, "one sweep over matrices of different kernels");
    if (items.size() >= (size_t(1) << 24)) fail(H2_EUNSUPPORTED, "GEMM batch above 2^24 items");
    int em = 64, en = 64;  // tile of the kernel that runs the batch
    variant = 0;
    if (amode >= 0) {
      if (prec < 0) fail(H2_EINVAL, "internal: GEMM batch without a precision");
      int max_m = 0;
      for (const GemmItem& it : items) max_m = std::max(max_m, int(it.M));
      variant = tune_gemm_variant(prec, role, amode, bmode, gemm_row_bucket(max_m));
      const int code = gemm_shape(prec, role, amode, bmode, variant);
      em = 16 * ((code >> 4) & 15);
      en = 16 * (code & 15);
    }
    // the solve sweeps give the row tiles of one tile column (the right-hand
    // sides) to the waves of one work-group, so that they read each S block
    // through one CU's cache: every item has the same rows there
    wg_rows = 1;
    if (role == ROLE_SOLVE && !items.empty()) {
      const int tm0 = (items[0].M + em - 1) / em;
      bool same = true;
      for (const GemmItem& it : items) same = same && (it.M + em - 1) / em == tm0;
      if (same) wg_rows = std::min(tm0, kSolveWaves);
    }
    for (size_t i = 0; i < items.size(); ++i) {
      const GemmItem& it = items[i];
      if (it.seg_end == it.seg_begin && mode != GEMM_STORE) continue;
      const int tm = (it.M + em - 1) / em, tn = (it.N + en - 1) / en;
      if (tm > 16 || tn > 16) fail(H2_EUNSUPPORTED, "GEMM item above 16 tiles along an edge");
      const int groups = (tm + wg_rows - 1) / wg_rows;  // tile rows of wg_rows row tiles
      for (int a = 0; a < groups; ++a)
        for (int b = 0; b < tn; ++b) tiles.push_back(int32_t((uint32_t(i) << 8) | (a << 4) | b));
    }
    ntiles = int32_t(tiles.size());
  }
  void drop_host() {
    std::vector<GemmItem>().swap(items);
    std::vector<GemmSeg>().swap(segs);
    std::vector<int32_t>().swap(tiles);
  }
  // Parameters of generated operands (kernel kind, as GemmItem::gkern) for every item.
  void set_generator(int dim, int kern, double scale, double diag, double param) {
    for (GemmItem& it : items) {
      it.gkern = uint8_t(kern);
      it.gdim = dim;
      it.gscale = scale;
      it.gdiag = diag;
      it.gparam = param;
    }
  }
  // Appends another batch's items and segments (same mode and role).
  void append(GemmBatch& o) {
    if (o.items.empty()) return;
    if (items.empty()) {
      mode = o.mode;
      role = o.role;
    }
    if (mode != o.mode || role != o.role) fail(H2_EINVAL, "internal: merging GEMM batches of another kind");
    const int32_t off = int32_t(segs.size());
    for (GemmItem it : o.items) {
      it.seg_begin += off;
      it.seg_end += off;
      items.push_back(it);
    }
    segs.insert(segs.end(), o.segs.begin(), o.segs.end());
    flops += o.flops;
    o.drop_host();
  }
  template <class T>
  void launch(hipStream_t st) const {
    if (ntiles <= 0) return;
    if (prec != (sizeof(T) == 4 ? 1 : 0) || gemm_shape(prec, role, amode, bmode, variant) == 0)
      fail(H2_EINVAL, "internal: GEMM batch launched in another precision or with a tile shape that is not built");
    GemmLaunch g{};
    g.amode = amode;
    g.bmode = bmode;
    g.items = d_items;
    g.segs = d_segs;
    g.tiles = d_tiles;
    g.ntiles = ntiles;
    g.mode = mode;
    g.role = role;
    g.kern = kern;
    g.variant = variant;
    g.wg_rows = wg_rows;
    launch_gemm<T>(g, st);
  }
};

// Raw host arrays to place in the same device allocation as the batches.
struct RawBlob {
  const void* host;
  size_t bytes;
  const void** dev;   // receives the device address
};

// Builds the tile lists, copies every batch's items, segments and tiles (and the
// extra blobs) into one device buffer `store`, and points the batches at it.
// The host arrays may be released on return.  With a copy stream the transfer
// runs there and `wait` (the compute stream) is made to wait for it, so that
// kernels already queued on `wait` keep running during the copy.
inline void upload_batches(const std::vector<GemmBatch*>& bs, DeviceBuffer& store,
                           const std::vector<RawBlob>& extra = {}, hipStream_t copy = nullptr,
                           hipStream_t wait = nullptr, bool parallel_pack = true) {
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  {
    int code = 0;
    std::string msg;
#pragma omp parallel for schedule(dynamic, 4) if (parallel_pack)
    for (long i = 0; i < long(bs.size()); ++i) {
      try {
        bs[i]->build_tiles();
      } catch (const Error& e) {
#pragma omp critical(h2_upload_error)
        if (!code) code = e.code, msg = e.msg;
      }
    }
    if (code) fail(code, msg);
  }
  size_t total = 0;
  std::vector<size_t> off(bs.size() * 3);
  for (size_t i = 0; i < bs.size(); ++i) {
    off[3 * i] = total;
    total = align(total + bs[i]->items.size() * sizeof(GemmItem));
    off[3 * i + 1] = total;
    total = align(total + bs[i]->segs.size() * sizeof(GemmSeg));
    off[3 * i + 2] = total;
    total = align(total + bs[i]->tiles.size() * sizeof(int32_t));
  }
  std::vector<size_t> xoff(extra.size());
  for (size_t i = 0; i < extra.size(); ++i) {
    xoff[i] = total;
    total = align(total + extra[i].bytes);
  }
  if (total == 0) return;
  if (trace_level() >= 2) std::fprintf(stderr, "[h2sp] upload: %zu GEMM batches, %.1f MB\n", bs.size(), total / 1e6);
  // page-locked staging, returned to the pool once the copy has completed
  struct Staging {
    PinnedBlock b;
    hipStream_t used = nullptr;  // stream of the copy out of it (drained before reuse)
    ~Staging() {
      if (used) (void)hipStreamSynchronize(used);
      pinned_release(b);
    }
  } stage{pinned_acquire(total)};
  char* staging = stage.b.ptr;
#pragma omp parallel for schedule(dynamic, 16) if (parallel_pack)
  for (long i = 0; i < long(bs.size()); ++i) {
    GemmBatch& b = *bs[i];
    if (!b.items.empty()) std::memcpy(&staging[off[3 * i]], b.items.data(), b.items.size() * sizeof(GemmItem));
    if (!b.segs.empty()) std::memcpy(&staging[off[3 * i + 1]], b.segs.data(), b.segs.size() * sizeof(GemmSeg));
    if (!b.tiles.empty()) std::memcpy(&staging[off[3 * i + 2]], b.tiles.data(), b.tiles.size() * sizeof(int32_t));
  }
  // blobs in pieces of at most 32 MiB, so that one large blob is copied by
  // many threads
  constexpr size_t kPiece = size_t(32) << 20;
  std::vector<std::pair<size_t, size_t>> pieces;  // (blob, first byte)
  for (size_t i = 0; i < extra.size(); ++i)
    for (size_t b = 0; b < extra[i].bytes; b += kPiece) pieces.emplace_back(i, b);
#pragma omp parallel for schedule(dynamic, 1) if (parallel_pack || pieces.size() > 8)
  for (long j = 0; j < long(pieces.size()); ++j) {
    const size_t i = pieces[j].first, b = pieces[j].second;
    const size_t n = std::min(kPiece, extra[i].bytes - b);
    std::memcpy(&staging[xoff[i] + b], static_cast<const char*>(extra[i].host) + b, n);
  }
  store.reset(total, copy);
  if (copy) {
    stage.used = copy;
    HIPCHECK(hipMemcpyAsync(store.ptr, staging, total, hipMemcpyHostToDevice, copy));
    hipEvent_t done;
    HIPCHECK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HIPCHECK(hipEventRecord(done, copy));
    HIPCHECK(hipStreamWaitEvent(wait, done, 0));
    HIPCHECK(hipStreamSynchronize(copy));  // the staging buffer is released below
    HIPCHECK(hipEventDestroy(done));
  } else {
    // on the current stream: a reused block may wait there for its last user
    stage.used = current_stream();
    HIPCHECK(hipMemcpyAsync(store.ptr, staging, total, hipMemcpyHostToDevice, current_stream()));
    HIPCHECK(hipStreamSynchronize(current_stream()));  // the staging buffer is released below
  }
  char* base = static_cast<char*>(store.ptr);
#pragma omp parallel for schedule(dynamic, 16) if (parallel_pack)
  for (long i = 0; i < long(bs.size()); ++i) {
    bs[i]->d_items = reinterpret_cast<const GemmItem*>(base + off[3 * i]);
    bs[i]->d_segs = reinterpret_cast<const GemmSeg*>(base + off[3 * i + 1]);
    bs[i]->d_tiles = reinterpret_cast<const int32_t*>(base + off[3 * i + 2]);
    bs[i]->drop_host();
  }
  for (size_t i = 0; i < extra.size(); ++i) *extra[i].dev = base + xoff[i];
}

// Bump allocation inside device memory the caller owns (no allocation of
// its own): pieces aligned to 256 bytes, H2_EINVAL once the region is used up.
struct DeviceArena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  const char* what = "scratch";
  void* take(size_t bytes) {
    const size_t at = (used + 255) & ~size_t(255);
    if (at > cap || bytes > cap - at)
      fail(H2_EINVAL, std::string(what) + ": needs more than its " + std::to_string(cap >> 20) + " MiB");
    used = at + bytes;
    return base + at;
  }
};

// As upload_batches, into a DeviceArena: staged through ordinary host memory
// and copied on stream st, which is synchronised before the host copy is
// released.  Allocates no device memory.
inline void upload_batches_into(const std::vector<GemmBatch*>& bs, DeviceArena& ar, hipStream_t st) {
  for (GemmBatch* b : bs) b->build_tiles();
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  size_t total = 0;
  std::vector<size_t> off(bs.size() * 3);
  for (size_t i = 0; i < bs.size(); ++i) {
    off[3 * i] = total;
    total = align(total + bs[i]->items.size() * sizeof(GemmItem));
    off[3 * i + 1] = total;
    total = align(total + bs[i]->segs.size() * sizeof(GemmSeg));
    off[3 * i + 2] = total;
    total = align(total + bs[i]->tiles.size() * sizeof(int32_t));
  }
  if (total == 0) return;
  char* base = static_cast<char*>(ar.take(total));
  std::vector<char> staging(total);
  for (size_t i = 0; i < bs.size(); ++i) {
    const GemmBatch& b = *bs[i];
    if (!b.items.empty()) std::memcpy(&staging[off[3 * i]], b.items.data(), b.items.size() * sizeof(GemmItem));
    if (!b.segs.empty()) std::memcpy(&staging[off[3 * i + 1]], b.segs.data(), b.segs.size() * sizeof(GemmSeg));
    if (!b.tiles.empty()) std::memcpy(&staging[off[3 * i + 2]], b.tiles.data(), b.tiles.size() * sizeof(int32_t));
  }
  HIPCHECK(hipMemcpyAsync(base, staging.data(), total, hipMemcpyHostToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));
  for (size_t i = 0; i < bs.size(); ++i) {
    bs[i]->d_items = reinterpret_cast<const GemmItem*>(base + off[3 * i]);
    bs[i]->d_segs = reinterpret_cast<const GemmSeg*>(base + off[3 * i + 1]);
    bs[i]->d_tiles = reinterpret_cast<const int32_t*>(base + off[3 * i + 2]);
    bs[i]->drop_host();
  }
}

}  // namespace h2
