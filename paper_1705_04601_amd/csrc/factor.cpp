// Block ILU(0) of S restricted to its own block pattern (the sparse
// factorisation step: a direct factorisation in Sections 5.3-5.4, an incomplete
// one as preconditioner in Section 5.5), in the symmetric form
// S ~ L D L^T, L^T_kj = Z_kj = D_k^{-1} S_kj (S is symmetric, Proposition 2.1),
// in the elimination order chosen at planning time (levels from the leaves up,
// greedy colours inside a level, so that rows of one colour are independent).
//
// Right-looking, scheduled by the levels of the elimination DAG (pivot k waits
// for every earlier k' with S_k'k stored).  Per DAG level, on the device:
//   1. D_k^{-1} for every pivot of the level (FP64 Gauss-Jordan, pivoting);
//   2. Z_kj = D_k^{-1} S_kj for the pivot rows (batched GEMM);
//   3. S_ij -= S_ki^T Z_kj for every stored target (i <= j) reached from a
//      pivot of the level, one work item per target, the pivots as K-segments
//      in elimination order (no atomics: the result is deterministic);
//   4. Z replaces the pivot rows of S.
// The levels are planned on the host, in order, by a producer thread (each level
// in parallel over its pivots); the calling thread uploads runs of planned
// levels on a copy stream and queues their launches, so host planning overlaps
// the device work of the levels before it.
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <mutex>
#include <thread>

#include <omp.h>

#include "factor.h"

namespace h2 {

namespace {

struct SchurRec {
  int64_t target;  // block number of (i, j)
  int64_t a_off;   // offset of S_ki in S
  int32_t z_off;   // offset of Z_kj in the Z buffer
  int32_t mk;
};

template <class T>
struct FactorLevel {
  std::vector<InvItem<T>> inv;
  std::vector<CopySeg> cps;
  std::vector<SchurItem> sitems;
  std::vector<SchurSeg> ssegs;
  std::vector<int32_t> stiles;
  const InvItem<T>* d_inv = nullptr;
  const CopySeg* d_cps = nullptr;
  const SchurItem* d_sitems = nullptr;
  const SchurSeg* d_ssegs = nullptr;
  const int32_t* d_stiles = nullptr;
  GemmBatch zb;
};

}  // namespace

template <class T>
static void factor_levels(h2_factor& f, hipStream_t st, double* phase_ms) {
  TraceTimer tt("factor");
  h2_sparse& sp = *f.sp;
  const i64 ncl = sp.ncl;
  const auto& mb = sp.nonbasis;
  T* S = sp.dS.as<T>();
  T* Inv = f.dInv.as<T>();
  const int dim = sp.H->tree.dim;
  auto cl = [&](i64 pos) { return sp.eorder[pos]; };
  std::vector<std::vector<i64>> by_level(f.nflev);
  for (i64 pos : f.rows) by_level[f.flev[pos]].push_back(pos);
  // Z buffer: largest level
  i64 zmax = 1;
  for (const auto& lv : by_level) {
    i64 z = 0;
    for (i64 pk : lv) {
      const i64 ck = cl(pk);
      for (i64 b = sp.rowptr[pk] + 1; b < sp.rowptr[pk + 1]; ++b) z += mb[ck] * mb[sp.colidx[b]];
    }
    zmax = std::max(zmax, z);
  }
  if (zmax >= (i64(1) << 31)) fail(H2_EUNSUPPORTED, "factor level too wide for 32-bit Z offsets");
  f.dZ.reset(sizeof(T) * zmax);
  T* Z = f.dZ.as<T>();
  // block number -> elimination position of its row
  std::vector<i64> row_of(sp.colidx.size());
  for (i64 pos = 0; pos < ncl; ++pos)
    for (i64 b = sp.rowptr[pos]; b < sp.rowptr[pos + 1]; ++b) row_of[b] = pos;

  std::vector<FactorLevel<T>> lvls(f.nflev);
  double fl_inv = 0, fl_z = 0, fl_s = 0;
  int too_wide = 0;
  // per-level completion flags of the planning, read by the uploading thread
  std::unique_ptr<std::atomic<int>[]> ready(new std::atomic<int>[f.nflev]);
  for (int lv = 0; lv < f.nflev; ++lv) ready[lv] = 0;
  std::mutex mu;
  std::condition_variable cv;
  const int nthr = std::max(1, omp_get_max_threads());
  std::vector<std::vector<i64>> marks(nthr);
  std::vector<std::vector<SchurRec>> local(nthr);
  std::vector<SchurRec> grouped;
  // Plans one level.  The pivots' Schur records are produced in parallel
  // (thread-local), spread over target buckets by sampled splitters, and each
  // bucket is sorted by (target, Z offset): Z offsets grow with the pivot's
  // elimination position, so every target's K-segments come in elimination
  // order whatever thread produced them.
  auto plan_level = [&](int lv) {
    FactorLevel<T>& L = lvls[lv];
    L.zb.role = ROLE_FACTOR;
    const std::vector<i64>& piv = by_level[lv];
    const long np = long(piv.size());
    std::vector<i64> zoffs(np), colbase(np + 1, 0);
    i64 zoff = 0;
    for (long q = 0; q < np; ++q) {
      const i64 pk = piv[q];
      const i64 ck = cl(pk);
      const i64 mk = mb[ck];
      const i64 dblk = sp.rowptr[pk];
      L.inv.push_back({S + sp.blk_off[dblk], Inv + f.inv_off[pk], int32_t(mk), 0});
      fl_inv += 2.0 * mk * mk * mk;
      zoffs[q] = zoff;
      const i64 b0 = dblk + 1, b1 = sp.rowptr[pk + 1];
      if (b0 == b1) continue;
      const i64 row_start = sp.blk_off[b0];
      i64 width = 0;
      for (i64 b = b0; b < b1; ++b) width += mb[sp.colidx[b]];
      for (i64 c0 = 0; c0 < width; c0 += 512) {
        const int w = int(std::min<i64>(512, width - c0));
        GemmItem& it = L.zb.item(int(mk), w, int(mk), w);
        GemmBatch::set_out(it, 0, Z + zoff + c0 * mk, mk, false);
        // D_k^{-1} is symmetric (D_k is): read it through its transpose so that
        // both operands run along K in memory
        L.zb.seg(Inv + f.inv_off[pk], int(mk), true, S + row_start + c0 * mk, int(mk), false, int(mk));
      }
      L.cps.push_back({row_start, zoff, mk * width});
      zoff += mk * width;
    }
    fl_z += L.zb.flops;
    // Schur targets (i, j), i before or equal to j, both in row k
    const int nt = int(std::min<long>(nthr, std::max<long>(1, np / 4)));
#pragma omp parallel num_threads(nt)
    {
      const int t = omp_get_thread_num();
      std::vector<SchurRec>& recs = local[t];
      recs.clear();
      std::vector<i64>& mark = marks[t];
      if (mark.empty()) mark.assign(ncl, -1);
#pragma omp for schedule(dynamic, 8)
      for (long q = 0; q < np; ++q) {
        const i64 pk = piv[q];
        const i64 mk = mb[cl(pk)];
        const i64 b0 = sp.rowptr[pk] + 1, b1 = sp.rowptr[pk + 1];
        i64 col = 0;
        for (i64 a = b0; a < b1; ++a) {
          const i64 pi = sp.epos[sp.colidx[a]];
          for (i64 b = sp.rowptr[pi]; b < sp.rowptr[pi + 1]; ++b) mark[sp.colidx[b]] = b;
          i64 col2 = col;
          for (i64 a2 = a; a2 < b1; ++a2) {
            const i64 s2 = sp.colidx[a2];
            const i64 tb = mark[s2];
            if (tb >= 0) recs.push_back({tb, sp.blk_off[a], int32_t(zoffs[q] + col2 * mk), int32_t(mk)});
            col2 += mb[s2];
          }
          for (i64 b = sp.rowptr[pi]; b < sp.rowptr[pi + 1]; ++b) mark[sp.colidx[b]] = -1;
          col += mb[sp.colidx[a]];
        }
      }
    }
    size_t total = 0;
    for (int t = 0; t < nt; ++t) total += local[t].size();
    auto by_target = [](const SchurRec& x, const SchurRec& y) {
      return x.target < y.target || (x.target == y.target && x.z_off < y.z_off);
    };
    // buckets of targets: splitters sampled from the records
    const int nbk = total < (size_t(1) << 15) ? 1 : 4 * nt;
    std::vector<i64> split;
    if (nbk > 1) {
      std::vector<i64> sample;
      const size_t stride = std::max<size_t>(1, total / (size_t(nbk) * 64));
      for (int t = 0; t < nt; ++t)
        for (size_t r = 0; r < local[t].size(); r += stride) sample.push_back(local[t][r].target);
      std::sort(sample.begin(), sample.end());
      for (int q = 1; q < nbk; ++q) split.push_back(sample[sample.size() * q / nbk]);
    }
    auto bucket_of = [&](i64 tb) { return int(std::upper_bound(split.begin(), split.end(), tb) - split.begin()); };
    std::vector<size_t> cnt(size_t(nt) * nbk, 0);  // [t][q]
#pragma omp parallel for num_threads(nt) schedule(static, 1)
    for (int t = 0; t < nt; ++t)
      for (const SchurRec& r : local[t]) ++cnt[size_t(t) * nbk + bucket_of(r.target)];
    std::vector<size_t> bstart(nbk + 1, 0), woff(size_t(nt) * nbk);
    {
      size_t o = 0;
      for (int q = 0; q < nbk; ++q) {
        bstart[q] = o;
        for (int t = 0; t < nt; ++t) {
          woff[size_t(t) * nbk + q] = o;
          o += cnt[size_t(t) * nbk + q];
        }
      }
      bstart[nbk] = o;
    }
    grouped.resize(total);
#pragma omp parallel for num_threads(nt) schedule(static, 1)
    for (int t = 0; t < nt; ++t) {
      size_t* w = &woff[size_t(t) * nbk];
      for (const SchurRec& r : local[t]) grouped[w[bucket_of(r.target)]++] = r;
    }
    // per bucket: sort, then items (one per target), segments (one per record,
    // written in place) and tiles
    L.ssegs.resize(total);
    std::vector<std::vector<SchurItem>> bitems(nbk);
    std::vector<std::vector<int32_t>> btiles(nbk);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1) reduction(+ : fl_s)
    for (int q = 0; q < nbk; ++q) {
      const size_t r0 = bstart[q], r1 = bstart[q + 1];
      std::sort(grouped.begin() + r0, grouped.begin() + r1, by_target);
      for (size_t r = r0; r < r1;) {
        const i64 tb = grouped[r].target;
        const i64 mi = mb[cl(row_of[tb])], mj = mb[sp.colidx[tb]];
        SchurItem si{sp.blk_off[tb], int32_t(mi), int32_t(mj), int32_t(r), 0};
        for (; r < r1 && grouped[r].target == tb; ++r) {
          L.ssegs[r] = {grouped[r].a_off, grouped[r].z_off, grouped[r].mk};
          fl_s += 2.0 * mi * mj * grouped[r].mk;
        }
        si.seg_end = int32_t(r);
        const uint32_t item = uint32_t(bitems[q].size());
        for (int a = 0; a < (mi + 63) / 64; ++a)
          for (int b = 0; b < (mj + 63) / 64; ++b) btiles[q].push_back(int32_t((item << 8) | (a << 4) | b));
        bitems[q].push_back(si);
      }
    }
    size_t nitems = 0, ntl = 0;
    for (int q = 0; q < nbk; ++q) {
      nitems += bitems[q].size();
      ntl += btiles[q].size();
    }
    if (nitems >= (size_t(1) << 24) || total >= (size_t(1) << 31)) {
      too_wide = 1;
      return;
    }
    L.sitems.reserve(nitems);
    L.stiles.reserve(ntl);
    for (int q = 0; q < nbk; ++q) {
      const uint32_t base = uint32_t(L.sitems.size());
      L.sitems.insert(L.sitems.end(), bitems[q].begin(), bitems[q].end());
      for (int32_t tcode : btiles[q]) L.stiles.push_back(int32_t(uint32_t(tcode) + (base << 8)));
    }
  };
  // plans the levels in order, each in parallel
  auto plan_all = [&]() {
    for (int lv = 0; lv < f.nflev && !too_wide; ++lv) {
      plan_level(lv);
      {
        std::lock_guard<std::mutex> lk(mu);
        ready[lv] = 1;
      }
      cv.notify_one();
    }
    std::vector<SchurRec>().swap(grouped);
    for (auto& v : local) std::vector<SchurRec>().swap(v);
    for (auto& v : marks) std::vector<i64>().swap(v);
    if (too_wide) fail(H2_EUNSUPPORTED, "Schur level above 2^24 targets or 2^31 segments");
  };
  std::vector<hipEvent_t> ev;
  auto mark_ev = [&]() {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    HIPCHECK(hipEventRecord(e, st));
    ev.push_back(e);
  };
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
    cv.notify_one();
  });
  hipStream_t cstream = nullptr;
  HIPCHECK(hipStreamCreateWithFlags(&cstream, hipStreamNonBlocking));  // no implicit sync with the null stream
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
        blobs.push_back({L.sitems.data(), L.sitems.size() * sizeof(SchurItem),
                         reinterpret_cast<const void**>(&L.d_sitems)});
        blobs.push_back({L.ssegs.data(), L.ssegs.size() * sizeof(SchurSeg),
                         reinterpret_cast<const void**>(&L.d_ssegs)});
        blobs.push_back({L.stiles.data(), L.stiles.size() * sizeof(int32_t),
                         reinterpret_cast<const void**>(&L.d_stiles)});
      }
      chunk_desc.emplace_back();
      upload_batches(all, chunk_desc.back(), blobs, cstream, st, /*parallel_pack=*/false);
      for (int lv = next; lv < end; ++lv) {
        FactorLevel<T>& L = lvls[lv];
        launch_inverse<T>(L.d_inv, int(L.inv.size()), f.dFlag.as<int>(), st);
        L.zb.template launch<T>(st, dim, 0.0, 0.0);
        mark_ev();
        SchurLaunch sl{L.d_sitems, L.d_ssegs, L.d_stiles, int32_t(L.stiles.size()), S, Z};
        launch_schur<T>(sl, st);
        mark_ev();
        launch_copy_segments<T>(L.d_cps, int(L.cps.size()), Z, S, st);
        std::vector<SchurItem>().swap(L.sitems);
        std::vector<SchurSeg>().swap(L.ssegs);
        std::vector<int32_t>().swap(L.stiles);
      }
      next = end;
    }
  } catch (...) {
    producer.join();
    (void)hipStreamDestroy(cstream);
    throw;
  }
  producer.join();
  HIPCHECK(hipStreamDestroy(cstream));
  if (perr) std::rethrow_exception(perr);
  if (int(ev.size()) != 2 * f.nflev + 1) fail(H2_EINVAL, "internal: factorisation stopped early");
  f.flops_inv += fl_inv;
  f.flops_z += fl_z;
  f.flops_schur += fl_s;
  tt.lap("plan+upload+enqueue");
  HIPCHECK(hipGetLastError());
  mark_ev();
  HIPCHECK(hipEventSynchronize(ev.back()));
  tt.lap("device-drain");
  double piv_ms = 0, schur_ms = 0;
  for (int lv = 0; lv < f.nflev; ++lv) {
    float a = 0, b = 0;
    HIPCHECK(hipEventElapsedTime(&a, ev[2 * lv], ev[2 * lv + 1]));
    HIPCHECK(hipEventElapsedTime(&b, ev[2 * lv + 1], ev[2 * lv + 2]));
    piv_ms += a;
    schur_ms += b;
  }
  float tot = 0;
  HIPCHECK(hipEventElapsedTime(&tot, ev.front(), ev.back()));
  for (auto e : ev) (void)hipEventDestroy(e);
  if (phase_ms) {
    phase_ms[4] = piv_ms;
    phase_ms[5] = schur_ms;
    phase_ms[6] = tot;
  }
}

h2_factor* factor(h2_sparse* sp, hipStream_t st, double* phase_ms) {
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
  f.dFlag.reset(sizeof(int));
  launch_fill_i(f.dFlag.as<int>(), 1, 0, st);
  if (sp->precision == H2_MIXED) factor_levels<float>(f, st, phase_ms);
  else factor_levels<double>(f, st, phase_ms);
  int flag = 0;
  HIPCHECK(hipMemcpy(&flag, f.dFlag.ptr, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) fail(H2_ESINGULAR, "singular pivot block in the factorisation of S");
  return fp.release();
}

}  // namespace h2
