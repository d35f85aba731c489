// Block ILU(0) of S restricted to its own block pattern (the sparse
// factorisation step: a direct factorisation in Sections 5.3-5.4, an incomplete
// one as preconditioner in Section 5.5), in the symmetric form
// S ~ L D L^T, L^T_kj = Z_kj = D_k^{-1} S_kj (S is symmetric, Proposition 2.1),
// in the elimination order chosen at planning time (levels from the leaves up,
// greedy colours inside a level, so that rows of one colour are independent).
//
// Left-looking (fan-in), scheduled by the levels of the elimination DAG (row i
// waits for every earlier k with S_ki stored).  Per DAG level, on the device:
//   1. Z_ki = D_k^{-1} S_ki for every stored S_ki above a row i of the level
//      (batched GEMM; row k and D_k^{-1} are final by then);
//   2. S_ij -= sum_k Z_ki^T S_kj for every stored target (i <= j) of the rows
//      of the level, one work item per target carrying all of its pivots k as
//      K-segments in elimination order, so each target is read and written
//      once (no atomics: the result is deterministic);
//   3. D_i^{-1} for every row of the level (FP64 Gauss-Jordan, pivoting);
//   4. Z_ki replaces S_ki (no later level reads S_ki: a later target (i', i)
//      would need S_i'i stored, which places i' before i in the DAG).
// At the end every stored block above the diagonal holds Z_kj and D_k^{-1} is
// in its own buffer, which is what the triangular solves read.
// The levels are planned on the host, in order, by a producer thread (each level
// in parallel over its rows); the calling thread uploads runs of planned levels
// on a copy stream and queues their launches, so host planning overlaps the
// device work of the levels before it.
#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <string>
#include <mutex>
#include <parallel/algorithm>
#include <thread>
#include <type_traits>

#include <omp.h>

#include "factor.h"

namespace h2 {

namespace {

template <class T>
struct FactorLevel {
  std::vector<InvItem<T>> inv;
  std::vector<CopySeg> cps;                 // Z_ki into the place of S_ki (end of the level)
  std::vector<CopySeg> zts, sts;            // Z_ki into tiles; the level's rows' blocks into tiles
  std::vector<DropItem> drops;              // ILUt: the level's rows' fill blocks and their thresholds
  std::vector<SchurItem> sitems;
  std::vector<int64_t> skeys;  // per item: tile-order key (host only)
  PodVector<SchurSeg> ssegs;
  PodVector<int32_t> sk;  // per segment: K without the padding of merged pivots (host only)
  std::vector<int32_t> stiles[kSchurClasses];  // Schur tiles by class (a launch each)
  std::vector<SchurReduce> reds;
  const InvItem<T>* d_inv = nullptr;
  const CopySeg* d_cps = nullptr;
  const CopySeg* d_zts = nullptr;
  const CopySeg* d_sts = nullptr;
  const DropItem* d_drops = nullptr;
  const SchurItem* d_sitems = nullptr;
  const SchurSeg* d_ssegs = nullptr;
  const int32_t* d_stiles[kSchurClasses] = {nullptr, nullptr, nullptr};
  const SchurReduce* d_reds = nullptr;
  GemmBatch zb;
  i64 zlen = 0;  // extent of the level's Z_ki blocks in the Z buffer
  int32_t nschur_tiles = 0, ntiles_cls[kSchurClasses] = {0, 0, 0};  // Schur tiles: all / by class
  double schur_flops = 0, cls_flops[kSchurClasses] = {0, 0, 0};      // Schur flops: all / by class
  double xcd_imbalance = 1;  // largest over mean work of the XCDs' tile ranges (traced)
  double col_share = 1, piv_share = 1;  // targets per distinct column, pivots per distinct pivot row (traced)
  double once_bytes = 0, stream_bytes = 0;  // Schur operands read once per level / once per tile (traced)
  std::string class_stats[kSchurClasses];   // the same by tile class (traced)
  double union2 = 1, union4 = 1;  // K of the union of the pivot lists of 2 / 4 consecutive targets over their sum (traced)
};

// Output of one chunk of rows of a level (concatenated in row order).
struct RowChunk {
  std::vector<SchurItem> items;
  std::vector<int64_t> keys;  // per item: tile-order key (row, place of the target column in space)
  PodVector<SchurSeg> segs;
  PodVector<int32_t> tk;  // per segment: K without the padding of merged pivots
  double flops = 0;
  double dense_pairs = 0;  // sum over rows of (pivots above the row) x (targets of the row)
};

}  // namespace

// level_events: time every level (pivots and Z, Schur update by tile class)
// with events; else only the whole factorisation (many small instances of a
// batch, where a few events per level cost more host time than their work).
template <class T>
static void factor_levels(h2_factor& f, hipStream_t st, double* phase_ms, bool level_events) {
  TraceTimer tt("factor");
  h2_sparse& sp = *f.sp;
  const i64 ncl = sp.ncl;
  const auto& mb = sp.nonbasis;
  T* S = sp.dS.as<T>();
  T* Inv = f.dInv.as<T>();
  auto cl = [&](i64 pos) { return sp.eorder[pos]; };
  std::vector<std::vector<i64>> by_level(f.nflev);
  for (i64 pos : f.rows) by_level[f.flev[pos]].push_back(pos);
  // column lists of the stored upper pattern: for S position i, the rows k
  // (elimination order) with S_ki stored and the block number of S_ki
  std::vector<i64> cptr(ncl + 1, 0), ck_pos, ck_blk;
  for (i64 pos = 0; pos < ncl; ++pos)
    for (i64 b = sp.rowptr[pos] + 1; b < sp.rowptr[pos + 1]; ++b) ++cptr[sp.epos[sp.colidx[b]] + 1];
  for (i64 i = 0; i < ncl; ++i) cptr[i + 1] += cptr[i];
  ck_pos.resize(cptr[ncl]);
  ck_blk.resize(cptr[ncl]);
  {
    std::vector<i64> fillp(cptr.begin(), cptr.end() - 1);
    for (i64 pos = 0; pos < ncl; ++pos)
      for (i64 b = sp.rowptr[pos] + 1; b < sp.rowptr[pos + 1]; ++b) {
        const i64 i = sp.epos[sp.colidx[b]];
        ck_pos[fillp[i]] = pos;
        ck_blk[fillp[i]++] = b;
      }
  }
  // Z buffers: the Z_ki blocks of the largest level, each with room for both
  // sides rounded up to 16: the pivot GEMMs write them column-major (ld m_k
  // rounded up to 16) into dZ, and the Schur kernel reads the copy in 16 x 16
  // tiles (launch_retile) in dZt, at the same offset
  auto kpad16 = [](i64 m) { return (m + 15) & ~i64(15); };
  i64 zmax = 1;
  for (const auto& lv : by_level) {
    i64 z = 0;
    for (i64 pi : lv)
      for (i64 c = cptr[pi]; c < cptr[pi + 1]; ++c) z += kpad16(mb[cl(ck_pos[c])]) * kpad16(mb[cl(pi)]);
    zmax = std::max(zmax, z);
  }
  if (zmax >= (i64(1) << 31)) fail(H2_EUNSUPPORTED, "factor level too wide for 32-bit Z offsets");
  f.dZ.reset(sizeof(T) * zmax);
  T* Z = f.dZ.as<T>();
  DeviceBuffer dZt(sizeof(T) * zmax);
  T* Zt = dZt.as<T>();
  // S_kj operands in tiles: every stored block above the diagonal gets a
  // tiled copy (both sides rounded up to 16) once its row is final, which the
  // Schur updates of later levels read instead of the block itself.  Used
  // when the copies fit in device memory (H2SP_SCHUR_TILED=0: never).  The
  // copies go in column order (for each S position j, its blocks S_kj in the
  // order of k), so that the blocks of consecutive pivots k of a column follow
  // each other along k, as the Z_ki of a row do in the Z buffer.
  // On a pattern extended by fill (exact mode, ILUt), a run of pivots whose
  // Z_ki and tiled S_kj blocks follow each other in memory is one segment
  // (the supernodal runs of the filled pattern): the tiles then go k-outer
  // and the S_kj copies in column order.  Otherwise one segment per pivot,
  // column-outer tiles and the copies in row order, which keeps the S_kj of
  // the tiles that run together (one pivot row, many targets) close in memory.
  // H2SP_SCHUR_MERGE=0 / =1 forces either.
  bool merge_runs = !sp.is_fill.empty();
  if (const char* e = std::getenv("H2SP_SCHUR_MERGE")) merge_runs = e[0] != '0';
  const bool kouter = merge_runs;
  std::vector<i64> st_off(sp.colidx.size(), -1);
  i64 st_len = 0;
  if (merge_runs) {
    for (i64 j = 0; j < ncl; ++j)
      for (i64 c = cptr[j]; c < cptr[j + 1]; ++c) {
        st_off[ck_blk[c]] = st_len;
        st_len += kpad16(mb[cl(ck_pos[c])]) * kpad16(mb[cl(j)]);
      }
  } else {
    for (i64 pos = 0; pos < ncl; ++pos)
      for (i64 b = sp.rowptr[pos] + 1; b < sp.rowptr[pos + 1]; ++b) {
        st_off[b] = st_len;
        st_len += kpad16(mb[cl(pos)]) * kpad16(mb[sp.colidx[b]]);
      }
  }
  bool tiled_s = st_len > 0;
  if (const char* e = std::getenv("H2SP_SCHUR_TILED")) tiled_s = tiled_s && e[0] != '0';
  if (tiled_s) {
    size_t free_b = 0, total_b = 0;
    HIPCHECK(hipMemGetInfo(&free_b, &total_b));
    free_b += cached_device_bytes();
    // leave room for the partial sums, the work lists and the solve after
    tiled_s = double(st_len) * sizeof(T) <= 0.8 * double(free_b) - double(sizeof(T)) * (double(zmax) + (1 << 25));
  }
  DeviceBuffer dSt;
  if (tiled_s) {
    try {
      dSt.reset(sizeof(T) * st_len, st);
    } catch (const Error& e) {
      if (e.code != H2_ENOMEM) throw;
      tiled_s = false;  // another factorisation took the memory meanwhile: read S in place
    }
  }
  T* St = tiled_s ? dSt.as<T>() : nullptr;
  f.schur_tiled = tiled_s;
  merge_runs = merge_runs && tiled_s;  // S_kj read in place: blocks of a column are not adjacent
  // end of each column list: the entries cptr[j] .. cend[j] - 1
  std::vector<i64> cend(cptr.begin() + 1, cptr.end());
  // per place in a column list: how many live entries from there on hold
  // consecutive elimination positions (runs of pivots); 0 marks an entry
  // whose block ILUt dropped (see prune_level)
  std::vector<int32_t> crun(merge_runs ? ck_pos.size() : 0);
  auto run_at = [&](i64 j, i64 c) -> int32_t {
    return (c + 1 < cend[j] && crun[c + 1] > 0 && ck_pos[c + 1] == ck_pos[c] + 1) ? crun[c + 1] + 1 : 1;
  };
  if (merge_runs)
    for (i64 j = 0; j < ncl; ++j)
      for (i64 c = cend[j] - 1; c >= cptr[j]; --c) crun[c] = run_at(j, c);
  // a dead entry is skipped by the plans (`live`)
  auto live = [&](i64 c) { return !merge_runs || crun[c] > 0; };
  // K of segment r without the padding rows of merged pivots
  auto seg_k = [&](const FactorLevel<T>& L, int32_t r) -> i64 { return merge_runs ? L.sk[r] : L.ssegs[r].K; };
  // ILUt: one flag per stored block (1 = dropped), written by the drop launches
  const bool ilut = !f.drop_thr2.empty();
  if (ilut && sp.colidx.size() >= (size_t(1) << 31)) fail(H2_EUNSUPPORTED, "ILUt pattern above 2^31 blocks");
  DeviceBuffer dDropFlag(ilut ? sp.colidx.size() : 0);
  // ILUt with planned runs: each level is planned after the previous level's
  // drop decisions are back on the host, and the dropped blocks (zero from
  // then on) leave the column lists, so that no later level multiplies them.
  // Planning then waits for the device level by level.  H2SP_ILUT_PRUNE=0
  // keeps the full structural fill in every plan.
  // (tau = 0 drops nothing: the plans then run ahead of the device as usual)
  bool prune = ilut && merge_runs && std::any_of(f.drop_thr2.begin(), f.drop_thr2.end(), [](double t) { return t > 0.0; });
  if (const char* e = std::getenv("H2SP_ILUT_PRUNE")) prune = prune && e[0] != '0';
  std::vector<uint8_t> hdrop(prune ? sp.colidx.size() : 0, 0);  // drop flags of finished levels
  int flags_done = -1;                                           // last level whose flags are in hdrop
  bool prod_abort = false;                                       // the enqueuing side failed
  auto is_dropped = [&](i64 b) { return f.drop_thr2[b] >= 0.0 && hdrop[b] != 0; };
  double prune_ms = 0, plan_ms = 0, flag_ms = 0;  // host time of the pruned planning (traced)
  // place of every stored block above the diagonal in its column list
  std::vector<i64> cidx(prune ? sp.colidx.size() : 0, -1);
  if (prune)
    for (i64 c = 0; c < i64(ck_blk.size()); ++c) cidx[ck_blk[c]] = c;
  // from a dead entry, a later entry on the way to the next live one (path
  // compressed by every lookup; the planning threads share it, so relaxed
  // atomics: any value written is a valid step)
  const i64 nent = i64(ck_pos.size());
  std::unique_ptr<std::atomic<i64>[]> nxt(new std::atomic<i64>[prune ? nent : 0]);
  for (i64 c = 0; c < (prune ? nent : 0); ++c) nxt[c].store(c + 1, std::memory_order_relaxed);
  // first live entry at or after c (nent past the last)
  auto next_live = [&](i64 c) {
    i64 r = c;
    while (r < nent && crun[r] == 0) r = nxt[r].load(std::memory_order_relaxed);
    for (i64 x = c; x < r && crun[x] == 0;) {
      const i64 y = nxt[x].load(std::memory_order_relaxed);
      nxt[x].store(r, std::memory_order_relaxed);
      x = y;
    }
    return r;
  };
  // marks the entries of the blocks that level l dropped as dead (a pivot row
  // k whose S_kj is zero from then on leaves the column list of j); only the
  // run lengths just before a dead entry change
  auto prune_level = [&](int l) {
    for (i64 pk : by_level[l])
      for (i64 b = sp.rowptr[pk] + 1; b < sp.rowptr[pk + 1]; ++b) {
        if (!is_dropped(b)) continue;
        const i64 j = sp.epos[sp.colidx[b]], c = cidx[b];
        crun[c] = 0;
        for (i64 q = c - 1; q >= cptr[j] && crun[q] > 0; --q) {
          const int32_t r = run_at(j, q);
          if (r == crun[q]) break;
          crun[q] = r;
        }
      }
  };
  // partial sums of split targets (at most pcap elements per level)
  f.pcap = std::min<i64>(i64(1) << 25, std::max<i64>(sp.s_entries, 1));
  f.dP.reset(sizeof(T) * f.pcap);
  T* Pbuf = f.dP.as<T>();

  std::vector<FactorLevel<T>> lvls(f.nflev);
  double fl_inv = 0, fl_z = 0, fl_s = 0;
  i64 nsplit = 0;
  int too_wide = 0;
  // per-level completion flags of the planning, read by the uploading thread
  std::unique_ptr<std::atomic<int>[]> ready(new std::atomic<int>[f.nflev]);
  for (int lv = 0; lv < f.nflev; ++lv) ready[lv] = 0;
  std::mutex mu;
  std::condition_variable cv;
  const int nthr = std::max(1, omp_get_max_threads());
  std::vector<std::vector<int32_t>> marks(nthr);
  // Split-K of long targets.  A level's Schur work is spread over about
  // kUnits tile-sized units where it has that much: a target whose K exceeds
  // 1.5 kt is cut at segment boundaries into parts of about kt, part 0
  // subtracting from S, the others storing partial sums that a reduction item
  // adds in part order (deterministic).  kt doubles until the partial sums of
  // the level fit the partial buffer.
  double shape_fl[4] = {0, 0, 0, 0}, pad_fl = 0, kpad = 0, ksum = 0;  // statistics (H2SP_TRACE)
  double st_pairs = 0, st_segs = 0, st_items = 0, st_rows = 0;
  constexpr int edge = schur_edge<T>;  // Schur tile edge
  double kUnits = 32768;  // H2SP_SCHUR_UNITS overrides
  if (const char* e = std::getenv("H2SP_SCHUR_UNITS")) kUnits = std::max(1.0, std::atof(e));

  // Levels of at least zpos_min tiles reorder their Schur tiles inside each
  // XCD's share; H2SP_SCHUR_ORDER=0 never does, =2 on every level.  The key
  // (H2SP_SCHUR_KEY): by default the target's row, then the first tree
  // position of its column cluster (targets of one row whose clusters are
  // close in space have close neighbours, so they share pivots); "z" orders
  // by the Z position where the tile's first segment starts.
  size_t zpos_min = size_t(tune_knob("schur.order_min", 16384));
  if (const char* e = std::getenv("H2SP_SCHUR_ORDER"))
    zpos_min = e[0] == '0' ? SIZE_MAX : e[0] == '2' ? 1 : zpos_min;
  bool key_z = tune_knob("schur.key_z", 0) != 0;
  if (const char* e = std::getenv("H2SP_SCHUR_KEY")) key_z = e[0] == 'z';
  const std::vector<i64>& tstart = sp.H->tree.start;
  i64 kMinK = tune_knob("schur.split_k", 512);  // smallest K of a part; H2SP_SCHUR_SPLIT_K overrides it
  // targets of class 2 (6 to 8 blocks of 16 along the longer side) as tiles of
  // half the edge (class 0) instead of one whole-target tile
  const bool split_big = tune_knob("schur.split_big", 0) != 0;
  if (const char* e = std::getenv("H2SP_SCHUR_SPLIT_K")) kMinK = std::max<i64>(1, std::atoll(e));
  const i64 pcap = f.pcap;
  auto split_targets = [&](const std::vector<SchurItem>& items, const std::vector<int64_t>& keys,
                           FactorLevel<T>& L) {
    const long ni = long(items.size());
    const bool par = ni > 16384;
    auto tiles_of = [&](const SchurItem& it) { return i64((it.M + edge - 1) / edge) * ((it.N + edge - 1) / edge); };
    double work = 0;
#pragma omp parallel for reduction(+ : work) schedule(static) num_threads(nthr) if (par)
    for (long t = 0; t < ni; ++t) work += double(items[t].ksum) * double(tiles_of(items[t]));
    if (trace_enabled()) {
      for (long t = 0; t < ni; ++t) {
        const SchurItem& it = items[t];
        const double k = it.ksum;
        shape_fl[(it.M > 64 ? 2 : 0) + (it.N > 64 ? 1 : 0)] += 2.0 * it.M * it.N * k;
        pad_fl += 2.0 * ((it.M + 15) / 16 * 16) * ((it.N + 15) / 16 * 16) * k;
        for (int32_t r = it.seg_begin; r < it.seg_end; ++r) kpad += (L.ssegs[r].K + 15) / 16 * 16;
        ksum += k;
      }
    }
    i64 kt = std::max<i64>(kMinK, i64(work / kUnits) + 1);
    auto parts_of = [&](long t) -> i64 {
      const i64 k = items[t].ksum;
      return k * 2 > 3 * kt ? (k + kt - 1) / kt : 1;
    };
    while (true) {
      i64 need = 0;
#pragma omp parallel for reduction(+ : need) schedule(static) num_threads(nthr) if (par)
      for (long t = 0; t < ni; ++t) need += (parts_of(t) - 1) * i64(items[t].M) * items[t].N;
      if (need <= pcap) break;
      kt *= 2;
    }
    // emission in contiguous ranges of items (in parallel), then merged in
    // range order with item indices and partial offsets shifted
    struct Out {
      std::vector<SchurItem> items;
      std::vector<int64_t> keys;
      std::vector<int32_t> tiles[kSchurClasses];
      std::vector<SchurReduce> reds;
      i64 pbase = 0, nsplit = 0;
      double cls_flops[kSchurClasses] = {0, 0, 0};
    };
    const int nparts = par ? 4 * nthr : 1;
    std::vector<Out> outs(nparts);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr) if (par)
    for (int p = 0; p < nparts; ++p) {
      Out& o = outs[p];
      auto emit = [&](const SchurItem& si, int64_t key) {
        const uint32_t item = uint32_t(o.items.size());
        o.keys.push_back(key);
        i64 k = 0;  // flops without the padding rows of merged pivots
        for (int32_t r = si.seg_begin; r < si.seg_end; ++r) k += seg_k(L, r);
        const bool half = split_big && schur_tile_class<T>(si.M, si.N, 0, 0) == 2;
        const int te = half ? edge / 2 : edge;
        for (int a = 0; a < (si.M + te - 1) / te; ++a)
          for (int b = 0; b < (si.N + te - 1) / te; ++b) {
            const int cls = schur_tile_class<T>(si.M, si.N, a * te, b * te, te);
            o.tiles[cls].push_back(schur_tile_code(item, a, b, half));
            o.cls_flops[cls] += 2.0 * std::min(te, si.M - a * te) * std::min(te, si.N - b * te) * double(k);
          }
        o.items.push_back(si);
      };
      for (long t = ni * p / nparts; t < ni * (p + 1) / nparts; ++t) {
        const SchurItem& it = items[t];
        const i64 np = parts_of(t);
        if (np == 1) {
          emit(it, keys[t]);
          continue;
        }
        const i64 len = i64(it.M) * it.N;
        int32_t begin = it.seg_begin;
        i64 acc = 0, part = 0;
        for (int32_t r = it.seg_begin; r < it.seg_end; ++r) {
          acc += L.ssegs[r].K;
          const bool last = r + 1 == it.seg_end;
          if (last || (part < np - 1 && acc * np >= (part + 1) * i64(it.ksum))) {
            SchurItem si = it;
            si.seg_begin = begin;
            si.seg_end = r + 1;
            if (part > 0) {
              si.partial = 1;
              si.out_off = o.pbase + (part - 1) * len;  // shifted by the range's base below
            }
            emit(si, keys[t]);
            begin = r + 1;
            ++part;
          }
        }
        if (part > 1) {
          o.reds.push_back({it.out_off, o.pbase, int32_t(len), int32_t(part - 1)});
          o.pbase += (part - 1) * len;
          ++o.nsplit;
        }
      }
    }
    std::vector<size_t> io(nparts + 1, 0), ro(nparts + 1, 0);
    std::vector<size_t> to[kSchurClasses];
    for (auto& v : to) v.assign(nparts + 1, 0);
    std::vector<i64> po(nparts + 1, 0);
    for (int p = 0; p < nparts; ++p) {
      io[p + 1] = io[p] + outs[p].items.size();
      for (int c = 0; c < kSchurClasses; ++c) to[c][p + 1] = to[c][p] + outs[p].tiles[c].size();
      ro[p + 1] = ro[p] + outs[p].reds.size();
      po[p + 1] = po[p] + outs[p].pbase;
      nsplit += outs[p].nsplit;
      for (int c = 0; c < kSchurClasses; ++c) L.cls_flops[c] += outs[p].cls_flops[c];
    }
    if (io[nparts] >= (size_t(1) << 24)) {
      too_wide = 1;
      return;
    }
    L.sitems.resize(io[nparts]);
    L.skeys.resize(io[nparts]);
    for (int c = 0; c < kSchurClasses; ++c) L.stiles[c].resize(to[c][nparts]);
    L.reds.resize(ro[nparts]);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthr) if (par)
    for (int p = 0; p < nparts; ++p) {
      const Out& o = outs[p];
      for (size_t i = 0; i < o.items.size(); ++i) {
        SchurItem si = o.items[i];
        if (si.partial) si.out_off += po[p];
        L.sitems[io[p] + i] = si;
        L.skeys[io[p] + i] = o.keys[i];
      }
      for (int c = 0; c < kSchurClasses; ++c)
        for (size_t i = 0; i < o.tiles[c].size(); ++i)
          L.stiles[c][to[c][p] + i] = int32_t(uint32_t(o.tiles[c][i]) + (uint32_t(io[p]) << 8));
      for (size_t i = 0; i < o.reds.size(); ++i) {
        SchurReduce r = o.reds[i];
        r.p_off += po[p];
        L.reds[ro[p] + i] = r;
      }
    }
  };
  // Schur work of a level on a filled pattern: for a target (i, j) the pivots
  // k with S_ki and S_kj stored are the intersection of the column lists of i
  // and j (both in elimination order), walked by runs of consecutive
  // positions with a binary search over the gaps.  A run is one segment (its
  // Z_ki follow each other in the Z buffer, its S_kj in the column-ordered
  // copies), and a segment whose blocks continue the previous one joins it.
  // A segment holds at most kcap padded rows (half the smallest split-K
  // part), so that long targets can still be split into parts that run in
  // parallel.  The rows are cut into pieces of targets, planned in parallel
  // and concatenated in row and target order: the same segments as one per
  // pivot joined afterwards, without visiting every pivot of every target.
  const i64 kcap = std::max<i64>(16, kMinK / 2);
  auto plan_runs = [&](const std::vector<i64>& rows, const std::vector<i64>& zbase, std::vector<RowChunk>& chunks) {
    const long nr = long(rows.size());
    i64 ntar = 0;
    for (long q = 0; q < nr; ++q) ntar += sp.rowptr[rows[q] + 1] - sp.rowptr[rows[q]];
    const i64 per = std::max<i64>(16, ntar / (16 * i64(nthr)) + 1);
    struct Piece {
      long q;
      i64 b0, b1;  // targets: stored blocks b0 .. b1 - 1 of row q
    };
    std::vector<Piece> pieces;
    for (long q = 0; q < nr; ++q) {
      const i64 t0 = sp.rowptr[rows[q]], t1 = sp.rowptr[rows[q] + 1];
      for (i64 b = t0; b < t1; b += per) pieces.push_back({q, b, std::min(t1, b + per)});
    }
    chunks.assign(pieces.size(), RowChunk());
#pragma omp parallel num_threads(nthr)
    {
      std::vector<i64> zo, kp, tp;  // per pivot of the row: Z offset, padded and true K before it
      long zrow = -1;
#pragma omp for schedule(dynamic, 1)
      for (long pc = 0; pc < long(pieces.size()); ++pc) {
        const Piece& P = pieces[pc];
        RowChunk& out = chunks[pc];
        const i64 pi = rows[P.q];
        const i64 mi = mb[cl(pi)], mi16 = kpad16(mi);
        const i64 c0 = cptr[pi], nci = cend[pi] - c0;
        const i64* ci = ck_pos.data() + c0;
        if (zrow != P.q) {
          zrow = P.q;
          zo.resize(nci + 1);
          kp.resize(nci + 1);
          tp.resize(nci + 1);
          zo[0] = zbase[P.q];
          kp[0] = tp[0] = 0;
          for (i64 p = 0; p < nci; ++p) {
            const i64 mk = live(c0 + p) ? mb[cl(ci[p])] : 0;  // dead entries take no room in Z
            zo[p + 1] = zo[p] + kpad16(mk) * mi16;
            kp[p + 1] = kp[p] + kpad16(mk);
            tp[p + 1] = tp[p] + mk;
          }
        }
        out.dense_pairs += double(nci) * double(P.b1 - P.b0);
        for (i64 b = P.b0; b < P.b1; ++b) {
          const i64 mj = mb[sp.colidx[b]], mj16 = kpad16(mj);
          const i64 cj0 = cptr[sp.epos[sp.colidx[b]]], ncj = cend[sp.epos[sp.colidx[b]]] - cj0;
          const i64* cj = ck_pos.data() + cj0;
          const size_t sb = out.segs.size();
          i64 p = 0, q = 0;
          while (p < nci && q < ncj) {
            if (crun[c0 + p] == 0) {  // S_ki dropped
              p = std::min(next_live(c0 + p), c0 + nci) - c0;
              continue;
            }
            if (crun[cj0 + q] == 0) {  // S_kj dropped
              q = std::min(next_live(cj0 + q), cj0 + ncj) - cj0;
              continue;
            }
            if (ci[p] < cj[q]) {
              p = std::lower_bound(ci + p + 1, ci + nci, cj[q]) - ci;
              continue;
            }
            if (ci[p] > cj[q]) {
              q = std::lower_bound(cj + q + 1, cj + ncj, ci[p]) - cj;
              continue;
            }
            // the run, in pieces of at most kcap padded rows (at least one
            // pivot each)
            const i64 e = p + std::min<i64>(crun[c0 + p], crun[cj0 + q]);
            while (p < e) {
              i64 u = std::upper_bound(kp.begin() + p + 1, kp.begin() + e + 1, kp[p] + kcap) - kp.begin() - 1;
              u = std::max(u, p + 1);
              const i64 K = kp[u - 1] - kp[p] + (tp[u] - tp[u - 1]);
              const i64 aoff = zo[p], boff = st_off[ck_blk[cj0 + q]];
              const int32_t tk = int32_t(tp[u] - tp[p]);
              q += u - p;
              p = u;
              if (out.segs.size() > sb) {
                SchurSeg& pv = out.segs.back();
                const i64 kpv = kpad16(pv.K);
                if (i64(pv.a_off) + kpv * mi16 == aoff && pv.b_off + kpv * mj16 == boff && kpv + K <= kcap) {
                  pv.K = int32_t(kpv + K);
                  out.tk.back() += tk;
                  continue;
                }
              }
              out.segs.push_back({boff, int32_t(aoff), int32_t(K)});
              out.tk.push_back(tk);
            }
          }
          if (out.segs.size() == sb) continue;
          SchurItem si{sp.blk_off[b], int32_t(mi), int32_t(mj), int32_t(sb), int32_t(out.segs.size()), 0, 0};
          i64 k = 0, kt = 0;
          for (size_t r = sb; r < out.segs.size(); ++r) {
            k += out.segs[r].K;
            kt += out.tk[r];
          }
          si.ksum = int32_t(k);
          out.flops += 2.0 * mi * mj * double(kt);
          out.items.push_back(si);
          out.keys.push_back((int64_t(P.q) << 32) | int64_t(tstart[sp.colidx[b]]));
        }
      }
    }
  };
  // Plans one level: Z GEMMs, copies and inverses row by row (cheap), Schur
  // targets in parallel over chunks of rows, concatenated in row order.
  auto plan_level = [&](int lv) {
    FactorLevel<T>& L = lvls[lv];
    L.zb.role = ROLE_FACTOR;
    L.zb.prec = sizeof(T) == 4 ? 1 : 0;
    const std::vector<i64>& rows = by_level[lv];
    const long nr = long(rows.size());
    std::vector<i64> zbase(nr + 1, 0);
    for (long q = 0; q < nr; ++q) {
      const i64 pi = rows[q];
      const i64 mi = mb[cl(pi)];
      L.inv.push_back({S + sp.blk_off[sp.rowptr[pi]], Inv + f.inv_off[pi], int32_t(mi), 0});
      fl_inv += 2.0 * mi * mi * mi;
      i64 z = zbase[q];
      for (i64 c = cptr[pi]; c < cend[pi]; ++c) {
        if (!live(c)) continue;  // S_ki dropped: Z_ki is zero and no plan reads it
        const i64 pk = ck_pos[c];
        const i64 mk = mb[cl(pk)];
        const i64 soff = sp.blk_off[ck_blk[c]];
        GemmItem& it = L.zb.item(int(mk), int(mi), int(mk), int(mi));
        GemmBatch::set_out(it, 0, Z + z, kpad16(mk), false);
        L.zts.push_back({z, z, int32_t(mk), int32_t(mi), int32_t(kpad16(mk)), kouter ? 1 : 0});
        // D_k^{-1} is symmetric (D_k is): read it through its transpose so that
        // both operands run along K in memory
        L.zb.seg(Inv + f.inv_off[pk], int(mk), true, S + soff, int(mk), false, int(mk));
        L.cps.push_back({soff, z, int32_t(mk), int32_t(mi), int32_t(kpad16(mk)), 0});
        z += kpad16(mk) * kpad16(mi);
      }
      zbase[q + 1] = z;
      // the row's fill blocks are tested against their threshold once the
      // level's update is done (ILUt)
      if (ilut)
        for (i64 b = sp.rowptr[pi] + 1; b < sp.rowptr[pi + 1]; ++b)
          if (f.drop_thr2[b] >= 0.0)
            L.drops.push_back({sp.blk_off[b], f.drop_thr2[b], int32_t(mi * mb[sp.colidx[b]]), int32_t(b)});
      // the row's blocks above the diagonal are final after this level
      if (tiled_s)
        for (i64 b = sp.rowptr[pi] + 1; b < sp.rowptr[pi + 1]; ++b)
          L.sts.push_back({st_off[b], sp.blk_off[b], int32_t(mi), int32_t(mb[sp.colidx[b]]), int32_t(mi), kouter ? 1 : 0});
    }
    L.zlen = zbase[nr];
    fl_z += L.zb.flops;
    // Schur targets: every stored (i, j), j at or after i, of a row i of the level
    int nchunk = int(std::min<long>(nr, 8L * nthr));
    int nt = int(std::min<long>(nthr, std::max<long>(1, nr / 2)));
    std::vector<RowChunk> chunks;
    if (merge_runs) {
      plan_runs(rows, zbase, chunks);
      nchunk = int(chunks.size());
      nt = nthr;
    } else {
      chunks.resize(nchunk);
#pragma omp parallel num_threads(nt)
    {
      std::vector<int32_t>& mark = marks[omp_get_thread_num()];
      if (mark.empty()) mark.assign(ncl, -1);
      std::vector<int32_t> cnt, fillp;
#pragma omp for schedule(dynamic, 1)
      for (int ch = 0; ch < nchunk; ++ch) {
        RowChunk& out = chunks[ch];
        const long q0 = nr * ch / nchunk, q1 = nr * (ch + 1) / nchunk;
        for (long q = q0; q < q1; ++q) {
          const i64 pi = rows[q];
          const i64 mi = mb[cl(pi)];
          const i64 t0 = sp.rowptr[pi], t1 = sp.rowptr[pi + 1];
          const int nt_row = int(t1 - t0);
          for (i64 b = t0; b < t1; ++b) mark[sp.colidx[b]] = int32_t(b - t0);
          cnt.assign(nt_row + 1, 0);
          for (i64 c = cptr[pi]; c < cend[pi]; ++c) {
            const i64 pk = ck_pos[c];
            for (i64 b = sp.rowptr[pk]; b < sp.rowptr[pk + 1]; ++b) {
              const int32_t t = mark[sp.colidx[b]];
              if (t >= 0) ++cnt[t + 1];
            }
          }
          for (int t = 0; t < nt_row; ++t) cnt[t + 1] += cnt[t];
          const size_t sbase = out.segs.size();
          out.segs.resize(sbase + cnt[nt_row]);
          fillp.assign(cnt.begin(), cnt.end() - 1);
          i64 zoff = zbase[q];
          for (i64 c = cptr[pi]; c < cend[pi]; ++c) {
            const i64 pk = ck_pos[c];
            const i64 mk = mb[cl(pk)];
            for (i64 b = sp.rowptr[pk]; b < sp.rowptr[pk + 1]; ++b) {
              const int32_t t = mark[sp.colidx[b]];
              if (t >= 0) out.segs[sbase + fillp[t]++] = {tiled_s ? st_off[b] : sp.blk_off[b], int32_t(zoff), int32_t(mk)};
            }
            zoff += kpad16(mk) * kpad16(mi);
          }
          for (i64 b = t0; b < t1; ++b) mark[sp.colidx[b]] = -1;
          out.dense_pairs += double(cend[pi] - cptr[pi]) * nt_row;
          for (int t = 0; t < nt_row; ++t) {
            if (cnt[t + 1] == cnt[t]) continue;
            const i64 mj = mb[sp.colidx[t0 + t]];
            SchurItem si{sp.blk_off[t0 + t], int32_t(mi), int32_t(mj), int32_t(sbase + cnt[t]),
                         int32_t(sbase + cnt[t + 1]), 0, 0};
            i64 k = 0;
            for (int32_t r = si.seg_begin; r < si.seg_end; ++r) k += out.segs[r].K;
            si.ksum = int32_t(k);
            out.flops += 2.0 * mi * mj * double(k);
            out.items.push_back(si);
            out.keys.push_back((int64_t(q) << 32) | int64_t(tstart[sp.colidx[t0 + t]]));
          }
        }
      }
    }
    }
    size_t nitems = 0, nsegs = 0;
    for (const RowChunk& c : chunks) {
      nitems += c.items.size();
      nsegs += c.segs.size();
      fl_s += c.flops;
      L.schur_flops += c.flops;
      st_pairs += c.dense_pairs;
    }
    st_segs += double(nsegs);
    st_items += double(nitems);
    st_rows += double(nr);
    if (nsegs >= (size_t(1) << 31)) {
      too_wide = 1;
      return;
    }
    std::vector<size_t> io(nchunk + 1, 0), so(nchunk + 1, 0);
    for (int ch = 0; ch < nchunk; ++ch) {
      io[ch + 1] = io[ch] + chunks[ch].items.size();
      so[ch + 1] = so[ch] + chunks[ch].segs.size();
    }
    std::vector<SchurItem> items(nitems);
    std::vector<int64_t> keys(nitems);
    L.ssegs.resize(nsegs);
    L.sk.resize(merge_runs ? nsegs : 0);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
    for (int ch = 0; ch < nchunk; ++ch) {
      RowChunk& c = chunks[ch];
      const int32_t sb = int32_t(so[ch]);
      for (size_t i = 0; i < c.items.size(); ++i) {
        SchurItem si = c.items[i];
        si.seg_begin += sb;
        si.seg_end += sb;
        items[io[ch] + i] = si;
        keys[io[ch] + i] = c.keys[i];
      }
      if (!c.segs.empty()) {
        std::memcpy(&L.ssegs[so[ch]], c.segs.data(), c.segs.size() * sizeof(SchurSeg));
        if (merge_runs) std::memcpy(&L.sk[so[ch]], c.tk.data(), c.tk.size() * sizeof(int32_t));
      }
      std::vector<SchurItem>().swap(c.items);
      std::vector<int64_t>().swap(c.keys);
      PodVector<SchurSeg>().swap(c.segs);
      PodVector<int32_t>().swap(c.tk);
    }
    split_targets(items, keys, L);
    if (L.sitems.size() >= (size_t(1) << 24)) too_wide = 1;
    // Inside each XCD's share of the tile list (the kernel gives XCD x the
    // x-th contiguous eighth, so the shares keep the work balance of target
    // order), tiles are reordered so that the tiles running at the same time
    // on one XCD read the same Z_ki blocks, which its L2 then serves to all of
    // them: by default by row and then by the place of the target's column
    // cluster in space, else by the Z position where the first segment starts.
    // Levels of fewer than 16384 tiles keep target order: there the planning
    // thread, not the kernel, sets the pace, and the sort would cost more than
    // it saves.  The order changes no result: every tile writes its own
    // output block, and partial sums are added by a later launch.
    // Each of the two tile lists (big and other tiles) is ordered this way.
    auto order_tiles = [&](std::vector<int32_t>& tl) {
      if (tl.size() < zpos_min || tl.size() >= (size_t(1) << 24)) return;
      const i64 n = i64(tl.size()), base = n / 8, rem = n % 8;
      std::vector<int64_t> ord(static_cast<size_t>(n));
#pragma omp parallel for schedule(static) num_threads(nthr) if (n > 65536)
      for (long q = 0; q < long(n); ++q) {
        const uint32_t item = uint32_t(tl[q]) >> 8;
        ord[q] = key_z ? (int64_t(L.ssegs[L.sitems[item].seg_begin].a_off) << 24) | int64_t(q)
                       : L.skeys[item];
      }
      std::vector<int32_t> idx(static_cast<size_t>(n));
      for (long q = 0; q < long(n); ++q) idx[q] = int32_t(q);
#pragma omp parallel for schedule(static) num_threads(std::min(nthr, 8)) if (n > 4096)
      for (int x = 0; x < 8; ++x) {
        const i64 b0 = x * base + std::min<i64>(x, rem), b1 = (x + 1) * base + std::min<i64>(x + 1, rem);
        std::stable_sort(idx.begin() + b0, idx.begin() + b1, [&](int32_t a, int32_t b) { return ord[a] < ord[b]; });
      }
      std::vector<int32_t> st(static_cast<size_t>(n));
#pragma omp parallel for schedule(static) num_threads(nthr) if (n > 65536)
      for (long q = 0; q < long(n); ++q) st[q] = tl[size_t(idx[q])];
      tl.swap(st);
    };
    for (auto& tl : L.stiles) order_tiles(tl);
    if (trace_level() >= 2) {
      // the kernel gives XCD x the x-th contiguous eighth of each tile list
      double w[8] = {0, 0, 0, 0, 0, 0, 0, 0}, tot = 0;
      for (const std::vector<int32_t>* tl : {&L.stiles[0], &L.stiles[1], &L.stiles[2]}) {
        const i64 n = i64(tl->size()), base = n / 8, rem = n % 8;
        for (int x = 0; x < 8; ++x)
          for (i64 t = x * base + std::min<i64>(x, rem); t < (x + 1) * base + std::min<i64>(x + 1, rem); ++t) {
            const uint32_t code = uint32_t((*tl)[t]);
            const SchurItem& it = L.sitems[code >> 8];
            const int m0 = int((code >> 4) & 15) * edge, n0 = int(code & 15) * edge;
            const double tm = std::min(edge, (it.M - m0 + 15) / 16 * 16), tn = std::min(edge, (it.N - n0 + 15) / 16 * 16);
            w[x] += tm * tn * it.ksum;
            tot += tm * tn * it.ksum;
          }
      }
      L.xcd_imbalance = *std::max_element(w, w + 8) / std::max(1e-30, tot / 8);
    }
    if (trace_level() >= 2) {
      std::vector<char> seen_j(ncl, 0), seen_k(ncl, 0);
      double nt = 0, nj = 0, np = 0, nk = 0;
      for (i64 pi : rows) {
        for (i64 b = sp.rowptr[pi]; b < sp.rowptr[pi + 1]; ++b) {
          ++nt;
          if (!seen_j[sp.colidx[b]]) seen_j[sp.colidx[b]] = 1, ++nj;
        }
        for (i64 c = cptr[pi]; c < cend[pi]; ++c) {
          ++np;
          if (!seen_k[ck_pos[c]]) seen_k[ck_pos[c]] = 1, ++nk;
        }
      }
      L.col_share = nt / std::max(1.0, nj);
      L.piv_share = np / std::max(1.0, nk);
      // pivot lists of consecutive targets of a row: how much would a group of
      // G targets sharing one pass over the union of their pivots do
      {
        double sum_k = 0, u2 = 0, u4 = 0;
        std::vector<int32_t> tpos(ncl, -1);
        for (i64 pi : rows) {
          const i64 t0 = sp.rowptr[pi], t1 = sp.rowptr[pi + 1];
          for (i64 b = t0; b < t1; ++b) tpos[sp.colidx[b]] = int32_t(b - t0);
          std::vector<char> g2, g4;
          for (i64 c = cptr[pi]; c < cend[pi]; ++c) {
            const i64 pk = ck_pos[c];
            const double mk = double(mb[cl(pk)]);
            g2.assign((t1 - t0) / 2 + 1, 0);
            g4.assign((t1 - t0) / 4 + 1, 0);
            for (i64 b = sp.rowptr[pk]; b < sp.rowptr[pk + 1]; ++b) {
              const int32_t t = tpos[sp.colidx[b]];
              if (t < 0) continue;
              sum_k += mk;
              if (!g2[t / 2]) g2[t / 2] = 1, u2 += 2 * mk;
              if (!g4[t / 4]) g4[t / 4] = 1, u4 += 4 * mk;
            }
          }
          for (i64 b = t0; b < t1; ++b) tpos[sp.colidx[b]] = -1;
        }
        L.union2 = u2 / std::max(1.0, sum_k);
        L.union4 = u4 / std::max(1.0, sum_k);
      }
      // operand bytes: every Z_ki and S_kj block once, targets read and
      // written once; against every tile reading its own operands
      std::vector<std::pair<i64, i64>> bb;
      bb.reserve(L.ssegs.size());
      double stream = 0;
      for (const SchurItem& it : L.sitems)
        for (int32_t r = it.seg_begin; r < it.seg_end; ++r) {
          const SchurSeg& sg = L.ssegs[r];
          bb.push_back({sg.b_off, i64(sg.K) * it.N});
          stream += double(sizeof(T)) * (double(kpad16(sg.K)) * it.M + double(sg.K) * it.N);
        }
      sort_range(bb.begin(), bb.end());
      double once = double(sizeof(T)) * double(L.zlen);
      for (size_t q = 0; q < bb.size(); ++q)
        if (q == 0 || bb[q].first != bb[q - 1].first) once += double(sizeof(T)) * double(bb[q].second);
      for (const SchurItem& it : L.sitems)
        if (!it.partial) once += 2.0 * sizeof(T) * double(it.M) * it.N;
      L.once_bytes = once;
      L.stream_bytes = stream;
      // the same split by tile class (big: more than 4 x 4 blocks of 16):
      // targets, flops, Z and S bytes streamed per tile and read once
      for (int c = 0; c < kSchurClasses; ++c) {
        double nt = 0, fl = 0, zs = 0, ss = 0, sm = 0, sn = 0, sk = 0, ns = 0;
        std::vector<std::pair<i64, i64>> za, sb;
        for (const SchurItem& it : L.sitems) {
          if (schur_tile_class<T>(it.M, it.N, 0, 0) != c) continue;
          ++nt;
          sm += it.M;
          sn += it.N;
          for (int32_t r = it.seg_begin; r < it.seg_end; ++r) {
            const SchurSeg& sg = L.ssegs[r];
            fl += 2.0 * it.M * it.N * seg_k(L, r);
            zs += double(sizeof(T)) * double(kpad16(sg.K)) * it.M;
            ss += double(sizeof(T)) * double(sg.K) * it.N;
            sk += sg.K;
            ++ns;
            za.push_back({sg.a_off, kpad16(sg.K) * it.M});
            sb.push_back({sg.b_off, i64(sg.K) * it.N});
          }
        }
        double zo = 0, so = 0;
        sort_range(za.begin(), za.end());
        sort_range(sb.begin(), sb.end());
        for (size_t q = 0; q < za.size(); ++q)
          if (q == 0 || za[q].first != za[q - 1].first) zo += double(sizeof(T)) * double(za[q].second);
        for (size_t q = 0; q < sb.size(); ++q)
          if (q == 0 || sb[q].first != sb[q - 1].first) so += double(sizeof(T)) * double(sb[q].second);
        char buf[320];
        std::snprintf(buf, sizeof(buf),
                      "%s: targets %.0f mean M %.1f N %.1f, segments %.0f mean K %.1f, %.4g GFLOP, "
                      "Z per tile %.3f GB once %.3f GB, S per tile %.3f GB once %.3f GB",
                      c == 0 ? "class 0" : c == 1 ? "class 1" : "class 2", nt, sm / std::max(1.0, nt),
                      sn / std::max(1.0, nt), ns,
                      sk / std::max(1.0, ns), fl / 1e9, zs / 1e9, zo / 1e9, ss / 1e9, so / 1e9);
        L.class_stats[c] = buf;
      }
    }
  };
  // plans the levels in order, each in parallel
  auto plan_all = [&]() {
    for (int lv = 0; lv < f.nflev && !too_wide; ++lv) {
      if (prune && lv > 0) {
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return flags_done >= lv - 1 || prod_abort; });
          if (prod_abort) break;
        }
        const auto t0 = std::chrono::steady_clock::now();
        prune_level(lv - 1);
        prune_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      }
      const auto t1 = std::chrono::steady_clock::now();
      plan_level(lv);
      if (prune) plan_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
      {
        std::lock_guard<std::mutex> lk(mu);
        ready[lv] = 1;
      }
      cv.notify_all();
    }
    for (auto& v : marks) std::vector<int32_t>().swap(v);
    if (too_wide) fail(H2_EUNSUPPORTED, "Schur level above 2^24 targets or 2^31 segments");
  };
  // events on the main stream: the start, then per level after the Z GEMMs,
  // after the Schur update (all classes joined) and at the level's end; per
  // level and tile class a start and an end event on the class's stream
  std::vector<hipEvent_t> ev, cev;
  auto new_ev = [&](std::vector<hipEvent_t>& v, hipStream_t s_) {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    v.push_back(e);  // owned (and destroyed) from here on, even if the record fails
    HIPCHECK(hipEventRecord(e, s_));
    return e;
  };
  auto mark_ev = [&]() { return new_ev(ev, st); };
  // events that only order the class streams after the level's Z (no timing)
  std::vector<hipEvent_t> sync_ev;
  auto sync_event = [&](hipStream_t s_) {
    hipEvent_t e;
    HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    sync_ev.push_back(e);
    HIPCHECK(hipEventRecord(e, s_));
    return e;
  };
  // per level and tile class: the index of its start event in cev, or -1
  // when the class has no tiles there (nothing launched, nothing timed)
  std::vector<std::array<int, kSchurClasses>> cls_at(f.nflev);
  // upload in runs of planned levels: as soon as the next level is ready,
  // every ready level after it (up to kMaxRun) goes in one copy
  constexpr int kMaxRun = 32;
  std::vector<DeviceBuffer> chunk_desc;
  chunk_desc.reserve(f.nflev);
  std::exception_ptr perr;
  bool done_planning = false;
  std::thread producer([&] {
    try {
      plan_all();
    } catch (...) {
      perr = std::current_exception();
    }
    std::lock_guard<std::mutex> lk(mu);
    done_planning = true;
    cv.notify_all();
  });
  // The tile classes of a level update disjoint targets: classes 1 and 2
  // run on streams of their own beside class 0 on the main stream, so that
  // the tail of one class's launch overlaps the others (all at the default
  // priority).
  hipStream_t cstream = nullptr, cls_st[kSchurClasses] = {st, nullptr, nullptr};
  auto destroy_streams = [&]() {
    if (cstream) (void)hipStreamDestroy(cstream);
    for (int c = 1; c < kSchurClasses; ++c)
      if (cls_st[c]) (void)hipStreamDestroy(cls_st[c]);
  };
  try {
    HIPCHECK(hipStreamCreateWithFlags(&cstream, hipStreamNonBlocking));  // no implicit sync with the null stream
    for (int c = 1; c < kSchurClasses; ++c) HIPCHECK(hipStreamCreateWithFlags(&cls_st[c], hipStreamNonBlocking));
  } catch (...) {
    destroy_streams();
    {
      std::lock_guard<std::mutex> lk(mu);
      prod_abort = true;
    }
    cv.notify_all();
    producer.join();
    throw;
  }
  mark_ev();
  try {
    int next = 0;
    while (next < f.nflev) {
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return ready[next] != 0 || done_planning; });
        if (!ready[next]) break;  // planning stopped early (error)
      }
      int end = next + 1;
      while (end < f.nflev && end - next < kMaxRun && ready[end]) ++end;
      std::vector<GemmBatch*> all;
      std::vector<RawBlob> blobs;
      for (int lv = next; lv < end; ++lv) {
        FactorLevel<T>& L = lvls[lv];
        all.push_back(&L.zb);
        blobs.push_back({L.inv.data(), L.inv.size() * sizeof(InvItem<T>), reinterpret_cast<const void**>(&L.d_inv)});
        blobs.push_back({L.cps.data(), L.cps.size() * sizeof(CopySeg), reinterpret_cast<const void**>(&L.d_cps)});
        blobs.push_back({L.zts.data(), L.zts.size() * sizeof(CopySeg), reinterpret_cast<const void**>(&L.d_zts)});
        blobs.push_back({L.sts.data(), L.sts.size() * sizeof(CopySeg), reinterpret_cast<const void**>(&L.d_sts)});
        blobs.push_back({L.drops.data(), L.drops.size() * sizeof(DropItem),
                         reinterpret_cast<const void**>(&L.d_drops)});
        blobs.push_back({L.sitems.data(), L.sitems.size() * sizeof(SchurItem),
                         reinterpret_cast<const void**>(&L.d_sitems)});
        blobs.push_back({L.ssegs.data(), L.ssegs.size() * sizeof(SchurSeg),
                         reinterpret_cast<const void**>(&L.d_ssegs)});
        for (int c = 0; c < kSchurClasses; ++c)
          blobs.push_back({L.stiles[c].data(), L.stiles[c].size() * sizeof(int32_t),
                           reinterpret_cast<const void**>(&L.d_stiles[c])});
        blobs.push_back({L.reds.data(), L.reds.size() * sizeof(SchurReduce),
                         reinterpret_cast<const void**>(&L.d_reds)});
      }
      chunk_desc.emplace_back();
      upload_batches(all, chunk_desc.back(), blobs, cstream, st, /*parallel_pack=*/false);
      for (int lv = next; lv < end; ++lv) {
        FactorLevel<T>& L = lvls[lv];
        L.zb.template launch<T>(st);
        launch_retile<T>(L.d_zts, int(L.zts.size()), Z, Zt, st);
        for (int c = 0; c < kSchurClasses; ++c) {
          L.ntiles_cls[c] = int32_t(L.stiles[c].size());
          L.nschur_tiles += L.ntiles_cls[c];
        }
        const bool fork_any = L.ntiles_cls[1] > 0 || L.ntiles_cls[2] > 0;
        hipEvent_t fork = nullptr;
        if (level_events) fork = mark_ev();
        else if (fork_any) fork = sync_event(st);
        cls_at[lv].fill(-1);
        for (int c = kSchurClasses - 1; c >= 0; --c) {
          if (L.ntiles_cls[c] == 0) continue;
          if (c > 0) HIPCHECK(hipStreamWaitEvent(cls_st[c], fork, 0));
          if (level_events) {
            cls_at[lv][c] = int(cev.size());
            new_ev(cev, cls_st[c]);
          }
          SchurLaunch sl{L.d_sitems, L.d_ssegs, L.d_stiles[c], int32_t(L.stiles[c].size()), S,
                         tiled_s ? St : S, Zt, Pbuf, tiled_s ? 1 : 0, kouter ? 1 : 0};
          launch_schur<T>(sl, c, cls_st[c]);
          const hipEvent_t done = level_events ? new_ev(cev, cls_st[c]) : (c > 0 ? sync_event(cls_st[c]) : nullptr);
          if (c > 0) HIPCHECK(hipStreamWaitEvent(st, done, 0));
        }
        if (level_events) mark_ev();
        launch_schur_reduce<T>(L.d_reds, int(L.reds.size()), Pbuf, S, st);
        // ILUt: the rows of the level are finished; small fill blocks go to zero
        // before anything reads them (tiled copies, Z of later levels, solves)
        if (ilut) launch_drop_small<T>(L.d_drops, int(L.drops.size()), S, dDropFlag.as<uint8_t>(), st);
        if (tiled_s) launch_retile<T>(L.d_sts, int(L.sts.size()), S, St, st);
        launch_inverse<T>(L.d_inv, int(L.inv.size()), f.dFlag.as<int>(), st);
        launch_copy_segments<T>(L.d_cps, int(L.cps.size()), Z, S, st);
        if (level_events) mark_ev();
        if (prune && lv + 1 < f.nflev) {
          // the level's drop flags, for the planning of the next level
          i64 b0 = i64(sp.colidx.size()), b1 = 0;
          for (i64 pk : by_level[lv]) {
            b0 = std::min(b0, sp.rowptr[pk] + 1);
            b1 = std::max(b1, sp.rowptr[pk + 1]);
          }
          const auto t0 = std::chrono::steady_clock::now();
          if (b1 > b0) {
            HIPCHECK(hipMemcpyAsync(hdrop.data() + b0, dDropFlag.as<uint8_t>() + b0, size_t(b1 - b0),
                                    hipMemcpyDeviceToHost, st));
            HIPCHECK(hipStreamSynchronize(st));
          }
          // the run's levels are done: their work lists can go back to the cache
          if (lv + 1 == end) chunk_desc.back() = DeviceBuffer();
          flag_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
          {
            std::lock_guard<std::mutex> lk(mu);
            flags_done = lv;
          }
          cv.notify_all();
        }
        std::vector<SchurItem>().swap(L.sitems);
        PodVector<SchurSeg>().swap(L.ssegs);
        for (auto& tl : L.stiles) std::vector<int32_t>().swap(tl);
        std::vector<SchurReduce>().swap(L.reds);
        std::vector<CopySeg>().swap(L.zts);
        std::vector<CopySeg>().swap(L.sts);
        std::vector<DropItem>().swap(L.drops);
      }
      next = end;
    }
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(mu);
      prod_abort = true;
    }
    cv.notify_all();
    producer.join();
    // the buffers of this call are freed in the order of the main stream:
    // let every queued launch finish first
    for (int c = 0; c < kSchurClasses; ++c) (void)hipStreamSynchronize(cls_st[c]);
    destroy_streams();
    for (auto e : ev) (void)hipEventDestroy(e);
    for (auto e : cev) (void)hipEventDestroy(e);
    for (auto e : sync_ev) (void)hipEventDestroy(e);
    throw;
  }
  producer.join();
  destroy_streams();  // work already queued on a destroyed stream still completes
  if (perr) std::rethrow_exception(perr);
  constexpr int kEv = 3;  // main-stream events per level (level_events)
  if (int(ev.size()) != (level_events ? kEv * f.nflev : 0) + 1) fail(H2_EINVAL, "internal: factorisation stopped early");
  f.flops_inv += fl_inv;
  f.flops_z += fl_z;
  f.flops_schur += fl_s;
  f.split_targets += nsplit;
  for (const auto& L : lvls) {
    f.schur_launches += L.nschur_tiles > 0 ? 1 : 0;
    for (int c = 0; c < kSchurClasses; ++c) {
      f.launches_cls[c] += L.ntiles_cls[c] > 0 ? 1 : 0;
      f.flops_cls[c] += L.cls_flops[c];
    }
  }
  tt.lap("plan+upload+enqueue");
  if (trace_enabled() && prune)
    std::fprintf(stderr, "[h2sp] ILUt pruned planning: prune %.1f ms, plan %.1f ms, wait for flags %.1f ms\n", prune_ms,
                 plan_ms, flag_ms);
  if (trace_enabled()) {
    const double tot = std::max(1.0, shape_fl[0] + shape_fl[1] + shape_fl[2] + shape_fl[3]);
    std::fprintf(stderr,
                 "[h2sp] schur flops by target shape (M<=64,N<=64 | M<=64,N>64 | M>64,N<=64 | M>64,N>64): "
                 "%.3f %.3f %.3f %.3f; 16-padded M N / exact %.3f; 16-padded K / exact %.3f; splits %lld\n",
                 shape_fl[0] / tot, shape_fl[1] / tot, shape_fl[2] / tot, shape_fl[3] / tot, pad_fl / tot,
                 kpad / std::max(1.0, ksum), (long long)nsplit);
    std::fprintf(stderr,
                 "[h2sp] schur pattern: rows %.0f targets %.0f segments %.0f (%.1f per target, mean K %.1f); "
                 "segments / (pivots x targets per row) %.3f\n",
                 st_rows, st_items, st_segs, st_segs / std::max(1.0, st_items), ksum / std::max(1.0, st_segs),
                 st_segs / std::max(1.0, st_pairs));
  }
  HIPCHECK(hipGetLastError());
  mark_ev();
  HIPCHECK(hipEventSynchronize(ev.back()));
  tt.lap("device-drain");
  if (ilut) {
    std::vector<uint8_t> flag(sp.colidx.size());
    HIPCHECK(hipMemcpy(flag.data(), dDropFlag.ptr, flag.size(), hipMemcpyDeviceToHost));
    for (size_t b = 0; b < flag.size(); ++b)
      if (f.drop_thr2[b] >= 0.0 && flag[b] < 2) (flag[b] ? f.ilut_dropped : f.ilut_kept) += 1;
  }
  double piv_ms = 0, schur_ms = 0, cls_ms[kSchurClasses] = {0, 0, 0};
  for (int lv = 0; level_events && lv < f.nflev; ++lv) {
    const hipEvent_t* e = &ev[size_t(kEv) * lv];
    float a = 0, c = 0, b = 0, bc[kSchurClasses] = {0, 0, 0};
    HIPCHECK(hipEventElapsedTime(&a, e[0], e[1]));
    HIPCHECK(hipEventElapsedTime(&b, e[1], e[2]));
    HIPCHECK(hipEventElapsedTime(&c, e[2], e[3]));
    for (int cls = 0; cls < kSchurClasses; ++cls) {
      const int k = cls_at[lv][cls];
      if (k < 0) continue;
      HIPCHECK(hipEventElapsedTime(&bc[cls], cev[k], cev[k + 1]));
      cls_ms[cls] += bc[cls];
    }
    piv_ms += a + c;
    schur_ms += b;
    if (trace_level() >= 2)
      std::fprintf(stderr,
                   "[h2sp] factor level %d: %zu rows, %d Schur tiles, %.4g GFLOP, %.3f ms (%.1f TF), XCD imbalance %.3f, "
                   "Z %.4f GB, rows per target column %.2f, rows per pivot %.2f, operands once %.3f GB, per tile %.3f GB, "
                   "grouped pivots x%.2f (2) x%.2f (4); "
                   "pivots and Z %.3f ms\n",
                   lv, by_level[lv].size(), lvls[lv].nschur_tiles, lvls[lv].schur_flops / 1e9, b,
                   lvls[lv].schur_flops / std::max(1e-6, double(b)) / 1e9, lvls[lv].xcd_imbalance,
                   double(lvls[lv].zlen) * sizeof(T) / 1e9, lvls[lv].col_share,
                   lvls[lv].piv_share, lvls[lv].once_bytes / 1e9, lvls[lv].stream_bytes / 1e9, lvls[lv].union2,
                   lvls[lv].union4, a + c);
    if (trace_level() >= 2)
      for (int k = 0; k < kSchurClasses; ++k)
        std::fprintf(stderr, "[h2sp] factor level %d tiles %.3f ms %s\n", lv, bc[k], lvls[lv].class_stats[k].c_str());
  }
  float tot = 0;
  HIPCHECK(hipEventElapsedTime(&tot, ev.front(), ev.back()));
  for (auto e : ev) (void)hipEventDestroy(e);
  for (auto e : cev) (void)hipEventDestroy(e);
  for (auto e : sync_ev) (void)hipEventDestroy(e);
  if (phase_ms) {
    phase_ms[4] = piv_ms;
    phase_ms[5] = schur_ms;
    phase_ms[6] = tot;
    for (int k = 0; k < kSchurClasses; ++k) phase_ms[7 + k] = cls_ms[k];
  }
}

// Exact mode: extends S's stored upper block pattern by the symbolic fill of
// its elimination in the elimination order (row structures of the block
// factor: a row's pattern is its own plus its children's in the elimination
// tree, the parent of a row being its first off-diagonal block), and re-lays
// S with the new blocks zero.  Block ILU(0) on the filled pattern is then the
// exact block factorisation.
// Row structures (positions after the row) of the block factor of S's
// pattern in elimination order.  Stops with ENOMEM once the entries counted
// exceed `budget` (when budget > 0).  entries / flops: stored entries of the
// filled upper triangle and 2 m_i m_j m_k summed over the Schur updates of
// the exact factorisation (i <= j both after pivot k in its row).
static std::vector<std::vector<i64>> symbolic_fill(const h2_sparse& sp, double budget, double elem_bytes,
                                                   double* entries, double* flops) {
  const i64 ncl = sp.ncl;
  const auto& mb = sp.nonbasis;
  double counted = 0, fl = 0;
  std::vector<std::vector<i64>> R(ncl), kids(ncl);
  std::vector<i64> mark(ncl, -1);
  for (i64 pos = 0; pos < ncl; ++pos) {
    if (mb[sp.eorder[pos]] == 0) {
      if (sp.rowptr[pos] != sp.rowptr[pos + 1]) fail(H2_EINVAL, "internal: S row without rows");
      continue;
    }
    std::vector<i64>& r = R[pos];
    mark[pos] = pos;
    for (i64 b = sp.rowptr[pos] + 1; b < sp.rowptr[pos + 1]; ++b) {
      const i64 j = sp.epos[sp.colidx[b]];
      if (mark[j] != pos) {
        mark[j] = pos;
        r.push_back(j);
      }
    }
    for (i64 c : kids[pos])
      for (i64 j : R[c])
        if (mark[j] != pos) {
          mark[j] = pos;
          r.push_back(j);
        }
    std::vector<i64>().swap(kids[pos]);
    std::sort(r.begin(), r.end());
    if (!r.empty()) kids[r[0]].push_back(pos);
    const double mk = double(mb[sp.eorder[pos]]);
    double sum = 0, sq = 0;
    for (i64 j : r) {
      const double mj = double(mb[sp.eorder[j]]);
      sum += mj;
      sq += mj * mj;
    }
    counted += mk * mk + mk * sum;
    fl += mk * (sum * sum + sq);  // 2 m_i m_j m_k over i < j, plus 2 m_i^2 m_k over i = j
    if (budget > 0 && counted > budget)
      fail(H2_ENOMEM, "exact factorisation: the filled S needs more than " +
                          std::to_string(counted * elem_bytes / 1e9) + " GB of device memory (" +
                          std::to_string(budget * elem_bytes / 1e9) + " GB usable)");
  }
  if (entries) *entries = counted;
  if (flops) *flops = fl;
  return R;
}

template <class T>
static void extend_by_fill(h2_sparse& sp, hipStream_t st) {
  TraceTimer tt("fill");
  const i64 ncl = sp.ncl;
  const auto& mb = sp.nonbasis;
  // device budget for the filled S: the symbolic pass stops as soon as the
  // entries counted so far exceed it (3D fill grows much faster than S)
  size_t free_b = 0, total_b = 0;
  HIPCHECK(hipMemGetInfo(&free_b, &total_b));
  free_b += cached_device_bytes();
  const double budget = std::max(1.0, 0.9 * double(free_b) / double(sizeof(T)));
  std::vector<std::vector<i64>> R = symbolic_fill(sp, budget, double(sizeof(T)), nullptr, nullptr);
  std::vector<i64> rowptr(ncl + 1, 0), colidx, blk_off;
  i64 ent = 0;
  for (i64 pos = 0; pos < ncl; ++pos) {
    const i64 c = sp.eorder[pos];
    if (mb[c] > 0) {
      colidx.push_back(c);
      blk_off.push_back(ent);
      ent += mb[c] * mb[c];
      for (i64 j : R[pos]) {
        const i64 cj = sp.eorder[j];
        colidx.push_back(cj);
        blk_off.push_back(ent);
        ent += mb[c] * mb[cj];
      }
    }
    rowptr[pos + 1] = i64(colidx.size());
    std::vector<i64>().swap(R[pos]);
  }
  tt.lap("symbolic");
  const size_t el = sizeof(T);
  // old blocks -> their places in the filled layout; every other block is fill
  std::vector<CopySeg> cps;
  cps.reserve(sp.colidx.size());
  std::vector<char> is_fill(colidx.size(), 1);
  for (i64 pos = 0; pos < ncl; ++pos) {
    const i64 mi = mb[sp.eorder[pos]];
    i64 nb = rowptr[pos];
    for (i64 b = sp.rowptr[pos]; b < sp.rowptr[pos + 1]; ++b) {
      const i64 cj = sp.colidx[b];
      while (nb < rowptr[pos + 1] && colidx[nb] != cj) ++nb;
      if (nb == rowptr[pos + 1]) fail(H2_EINVAL, "internal: fill pattern misses a block of S");
      cps.push_back({blk_off[nb], sp.blk_off[b], int32_t(mi), int32_t(mb[cj]), int32_t(mi), 0});
      is_fill[nb] = 0;
    }
  }
  DeviceBuffer nS(el * size_t(std::max<i64>(ent, 1)));
  if constexpr (std::is_same<T, float>::value) launch_fill_f(nS.as<float>(), ent, 0.0f, st);
  else launch_fill(nS.as<double>(), ent, 0.0, st);
  DeviceBuffer dcps(sizeof(CopySeg) * std::max<size_t>(cps.size(), 1));
  HIPCHECK(hipMemcpyAsync(dcps.ptr, cps.data(), sizeof(CopySeg) * cps.size(), hipMemcpyHostToDevice, st));
  launch_copy_segments<T>(dcps.as<CopySeg>(), int(cps.size()), sp.dS.as<T>(), nS.as<T>(), st);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(st));
  sp.dS = std::move(nS);
  sp.rowptr.swap(rowptr);
  sp.colidx.swap(colidx);
  sp.blk_off.swap(blk_off);
  sp.is_fill.swap(is_fill);
  sp.s_entries = ent;
  tt.lap("relayout");
}

void analyze_fill(const h2_sparse& sp, double* entries, double* flops) {
  (void)symbolic_fill(sp, 0.0, double(sp.elem), entries, flops);
}

// Square of the ILUt drop threshold of every fill block: (tau ||S_i,:||_F)^2
// for block row i, the norm over both triangles of S as given (before any
// update; the fill blocks are zero then).  The block norms are taken on the
// device.
template <class T>
static std::vector<double> drop_thresholds(const h2_sparse& sp, double tau, hipStream_t st) {
  const i64 nb = i64(sp.colidx.size());
  std::vector<BlockRef> refs(nb);
  std::vector<i64> row_of(nb);
  for (i64 pos = 0; pos < sp.ncl; ++pos)
    for (i64 b = sp.rowptr[pos]; b < sp.rowptr[pos + 1]; ++b) {
      refs[b] = {sp.blk_off[b], i64(sp.nonbasis[sp.eorder[pos]]) * sp.nonbasis[sp.colidx[b]]};
      row_of[b] = pos;
    }
  DeviceBuffer drefs(sizeof(BlockRef) * std::max<i64>(nb, 1)), dsq(sizeof(double) * std::max<i64>(nb, 1));
  HIPCHECK(hipMemcpyAsync(drefs.ptr, refs.data(), sizeof(BlockRef) * nb, hipMemcpyHostToDevice, st));
  launch_block_sumsq<T>(drefs.as<BlockRef>(), int(nb), sp.dS.as<T>(), dsq.as<double>(), st);
  HIPCHECK(hipGetLastError());
  std::vector<double> sq(nb);
  HIPCHECK(hipMemcpyAsync(sq.data(), dsq.ptr, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  std::vector<double> row2(sp.ncl, 0.0);  // by elimination position, in block order
  for (i64 b = 0; b < nb; ++b) {
    row2[row_of[b]] += sq[b];
    if (b != sp.rowptr[row_of[b]]) row2[sp.epos[sp.colidx[b]]] += sq[b];  // the mirror block
  }
  std::vector<double> thr2(nb, -1.0);
  for (i64 b = 0; b < nb; ++b)
    if (sp.is_fill[b]) {
      const double t = tau * std::sqrt(row2[row_of[b]]);
      thr2[b] = t * t;
    }
  return thr2;
}

h2_factor* factor(h2_sparse* sp, int mode, double tau, hipStream_t st, double* phase_ms, bool level_events) {
  if (mode == H2_FACTOR_EXACT || mode == H2_FACTOR_ILUT) {
    if (sp->precision == H2_MIXED) extend_by_fill<float>(*sp, st);
    else extend_by_fill<double>(*sp, st);
  }
  sp->factored = true;
  auto fp = std::make_unique<h2_factor>();
  h2_factor& f = *fp;
  f.sp = sp;
  const i64 ncl = sp->ncl;
  const auto& mb = sp->nonbasis;
  f.flev.assign(ncl, -1);
  f.blev.assign(ncl, -1);
  f.inv_off.assign(ncl, -1);
  std::vector<std::vector<i64>> col(ncl);
  i64 io = 0;
  for (i64 pos = 0; pos < ncl; ++pos) {
    const i64 c = sp->eorder[pos];
    if (mb[c] == 0) continue;
    f.rows.push_back(pos);
    if (sp->rowptr[pos] == sp->rowptr[pos + 1] || sp->colidx[sp->rowptr[pos]] != c)
      fail(H2_EINVAL, "internal: missing diagonal block of S");
    f.inv_off[pos] = io;
    io += mb[c] * mb[c];
    for (i64 b = sp->rowptr[pos] + 1; b < sp->rowptr[pos + 1]; ++b) col[sp->epos[sp->colidx[b]]].push_back(pos);
  }
  for (i64 pos : f.rows) {
    int l = 0;
    for (i64 k : col[pos]) l = std::max(l, f.flev[k] + 1);
    f.flev[pos] = l;
    f.nflev = std::max(f.nflev, l + 1);
  }
  for (auto it = f.rows.rbegin(); it != f.rows.rend(); ++it) {
    const i64 pos = *it;
    int l = 0;
    for (i64 b = sp->rowptr[pos] + 1; b < sp->rowptr[pos + 1]; ++b)
      l = std::max(l, f.blev[sp->epos[sp->colidx[b]]] + 1);
    f.blev[pos] = l;
    f.nblev = std::max(f.nblev, l + 1);
  }
  f.dInv.reset(sp->elem * std::max<i64>(io, 1));
  if (mode == H2_FACTOR_ILUT)
    f.drop_thr2 = sp->precision == H2_MIXED ? drop_thresholds<float>(*sp, tau, st) : drop_thresholds<double>(*sp, tau, st);
  f.dFlag.reset(sizeof(int));
  launch_fill_i(f.dFlag.as<int>(), 1, 0, st);
  if (sp->precision == H2_MIXED) factor_levels<float>(f, st, phase_ms, level_events);
  else factor_levels<double>(f, st, phase_ms, level_events);
  int flag = 0;
  HIPCHECK(hipMemcpy(&flag, f.dFlag.ptr, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) fail(H2_ESINGULAR, "singular pivot block in the factorisation of S");
  return fp.release();
}

}  // namespace h2
