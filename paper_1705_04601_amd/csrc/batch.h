// Host-side builder of batched GEMM launches (items, K-segments, tile list).
#pragma once

#include <algorithm>
#include <vector>

#include "h2_internal.h"
#include "kernels.h"

namespace h2 {

// Work list of one batched GEMM launch, kept on the device for replay.
struct GemmBatch {
  std::vector<GemmItem> items;
  std::vector<GemmSeg> segs;
  std::vector<int32_t> tiles;
  DeviceBuffer d_items, d_segs, d_tiles;
  int mode = GEMM_STORE;
  int role = ROLE_TRANSFORM;
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
  // Builds the tile list and copies everything to the device.
  void finalize() {
    tiles.clear();
    if (items.size() >= (size_t(1) << 24)) fail(H2_EUNSUPPORTED, "GEMM batch above 2^24 items");
    for (size_t i = 0; i < items.size(); ++i) {
      const GemmItem& it = items[i];
      if (it.seg_end == it.seg_begin && mode != GEMM_STORE) continue;
      const int tm = (it.M + 31) / 32, tn = (it.N + 31) / 32;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b) tiles.push_back(int32_t((uint32_t(i) << 8) | (a << 4) | b));
    }
    d_items = upload(items);
    d_segs = upload(segs);
    d_tiles = upload(tiles);
  }
  // Releases the host copies once on the device.
  void drop_host() {
    std::vector<GemmItem>().swap(items);
    std::vector<GemmSeg>().swap(segs);
  }
  template <class T>
  void launch(hipStream_t st, int dim, double scale, double diag) const {
    if (tiles.empty()) return;
    GemmLaunch g{};
    g.items = d_items.as<GemmItem>();
    g.segs = d_segs.as<GemmSeg>();
    g.tiles = d_tiles.as<int32_t>();
    g.ntiles = int32_t(tiles.size());
    g.mode = mode;
    g.role = role;
    g.dim = dim;
    g.scale = scale;
    g.diag = diag;
    launch_gemm<T>(g, st);
  }
};

}  // namespace h2
