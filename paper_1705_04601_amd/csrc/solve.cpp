// Solve of A x = b through S y = U^T b, x = V y (eq. sp0), with the block
// ILU(0) of S as the S-solver and iterative refinement against the FP64 H^2
// matrix-vector product:  x += V (L D L^T)^{-1} U^T r,  r = b - A_H2 x.
//
// U^T sweep (leaves -> root): w = Q_t^T z_t, rows k_t.. go to y (S order),
// rows ..k_t to the father's z.  V sweep (root -> leaves): z_t = Q_t [z_t^b; y_t].
// Triangular solves by the levels of the elimination DAG: forward
// u_i = r_i - sum_k Z_ki^T u_k, diagonal v_i = D_i^{-1} u_i, backward
// x_i = v_i - sum_j Z_ij x_j.
// Blocks of right-hand sides are stored RHS-fastest (element (i, j) at
// i nrhs + j) and every product is formed transposed (C^T = B^T A^T), so that
// the right-hand sides run along the rows of each output tile: loads of them
// and stores are contiguous, and a block of rows is one contiguous piece.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "factor.h"

namespace h2 {

struct MatvecPlan;
MatvecPlan& matvec_plan(const h2_matrix& H, i64 nrhs);
void run_matvec_tree(const h2_matrix& H, MatvecPlan& p, hipStream_t st);
struct MatvecPlanView {
  double* xt;
  double* yt;
};
MatvecPlanView matvec_buffers(MatvecPlan& p);

// With an arena the vectors and the work lists are placed in it (no device
// allocation) and the plan is launched eagerly; else they get buffers of
// their own and the application is captured as a graph on first use.
template <class T>
static std::unique_ptr<SolvePlan> make_solve_plan(h2_factor& f, i64 nrhs, DeviceArena* arena = nullptr) {
  TraceTimer tt("solve-plan");
  h2_sparse& sp = *f.sp;
  h2_matrix& H = *sp.H;
  const Tree& tr = H.tree;
  const i64 n = tr.n, ncl = sp.ncl;
  const int L = tr.depth;
  auto p = std::make_unique<SolvePlan>();
  p->nrhs = nrhs;
  p->tune_gen = tune_generation();
  const auto& na = sp.n_act;
  const auto& kp = sp.kept;
  const auto& mb = sp.nonbasis;
  // z slots for non-leaf clusters
  std::vector<i64> zoff(ncl, -1);
  i64 zs = 0;
  for (i64 c = 0; c < tr.first_at_level(0); ++c)
    if (na[c] > 0) {
      zoff[c] = zs;
      zs += na[c] * nrhs;
    }
  T *zin, *zb, *y, *w;
  if (arena) {
    p->eager = true;
    zin = static_cast<T*>(arena->take(sizeof(T) * n * nrhs));
    zb = static_cast<T*>(arena->take(sizeof(T) * std::max<i64>(zs, 1)));
    y = static_cast<T*>(arena->take(sizeof(T) * n * nrhs));
    w = static_cast<T*>(arena->take(sizeof(T) * n * nrhs));
    p->rs_ptr = static_cast<double*>(arena->take(sizeof(double) * n * nrhs));
  } else {
    p->zin.reset(sizeof(T) * n * nrhs);       // right-hand side in tree order (leaf z)
    p->zbuf.reset(sizeof(T) * std::max<i64>(zs, 1));
    p->y.reset(sizeof(T) * n * nrhs);
    p->w.reset(sizeof(T) * n * nrhs);
    p->rs.reset(sizeof(double) * n * nrhs);
    p->colscale.reset(sizeof(double) * nrhs);
    zin = p->zin.as<T>();
    zb = p->zbuf.as<T>();
    y = p->y.as<T>();
    w = p->w.as<T>();
    p->rs_ptr = p->rs.as<double>();
  }
  p->zin_ptr = zin;
  const T* Q = (sp.precision == H2_MIXED) ? sp.dQt.as<T>() : reinterpret_cast<const T*>(sp.dQ.as<double>());
  const T* S = sp.dS.as<T>();
  // Operands of the backward sweep, when the tuning table asks: every block
  // of S transposed (made once per factor, when it fits in a third of the
  // memory the device can give), so that the backward sweep reads
  // K-contiguous blocks like the forward one instead of strided ones.  Off by
  // default: on the 1M-point cube it takes 7 ms off an application (239 vs
  // 246 ms) and costs a pass over S per factor.
  const T* ST = nullptr;
  if (!arena && tune_knob("solve.transpose", 0) != 0) {
    if (!f.st_tried) {
      f.st_tried = true;
      const size_t bytes = sizeof(T) * size_t(std::max<i64>(sp.s_entries, 1));
      size_t free_b = 0, total_b = 0;
      HIPCHECK(hipMemGetInfo(&free_b, &total_b));
      if (bytes <= (free_b + cached_device_bytes()) / 3) {
        std::vector<CopySeg> segs;
        for (i64 pos = 0; pos < ncl; ++pos) {
          const int rows = int(mb[sp.eorder[pos]]);
          for (i64 b = sp.rowptr[pos]; b < sp.rowptr[pos + 1]; ++b) {
            const int cols = int(mb[sp.colidx[b]]);
            if (rows > 0 && cols > 0) segs.push_back({sp.blk_off[b], sp.blk_off[b], rows, cols, rows, 0});
          }
        }
        f.dST.reset(bytes);
        DeviceBuffer dsegs(sizeof(CopySeg) * std::max<size_t>(segs.size(), 1));
        HIPCHECK(hipMemcpyAsync(dsegs.ptr, segs.data(), sizeof(CopySeg) * segs.size(), hipMemcpyHostToDevice,
                                current_stream()));
        launch_transpose_blocks<T>(dsegs.as<CopySeg>(), int(segs.size()), S, f.dST.as<T>(), current_stream());
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(current_stream()));
      }
    }
    if (f.dST.ptr) ST = f.dST.as<T>();
  }
  (void)0;
  const T* Inv = f.dInv.as<T>();
  auto son_off = [&](i64 c) -> i64 { return (c % 2 == 1) ? 0 : kp[c - 1]; };
  auto zslot = [&](i64 c) -> T* { return tr.is_leaf(c) ? zin + tr.start[c] * nrhs : zb + zoff[c]; };
  const int N = int(nrhs);
  // U^T sweep: w^T = z_t^T Q_t, columns ..k_t to the father's slot, the rest to y
  p->up.resize(L + 1);
  for (int k = 0; k <= L; ++k) {
    for (i64 c = tr.first_at_level(k); c < tr.first_at_level(k) + tr.count_at_level(k); ++c) {
      if (na[c] == 0) continue;
      GemmItem& it = p->up[k].item(N, int(na[c]), N, int(kp[c]));
      if (kp[c] > 0) GemmBatch::set_out(it, 0, zslot((c - 1) / 2) + son_off(c) * nrhs, nrhs, false);
      if (mb[c] > 0) GemmBatch::set_out(it, 1, y + sp.soff[c] * nrhs, nrhs, false);
      p->up[k].seg(zslot(c), N, false, Q + sp.q_off[c], int(na[c]), false, int(na[c]));
    }
  }
  // forward and backward triangular solves, right-looking by DAG level: once
  // the rows of a level are final they update every row they reach; each work
  // item owns one target row and takes the level's contributions in
  // elimination order (short chains, many items per launch).  Levels are
  // planned in parallel.
  std::vector<std::vector<i64>> fl(f.nflev), bl(f.nblev);
  for (i64 pos : f.rows) {
    fl[f.flev[pos]].push_back(pos);
    bl[f.blev[pos]].push_back(pos);
  }
  std::vector<i64> row_of(sp.colidx.size());
  for (i64 pos = 0; pos < ncl; ++pos)
    for (i64 b = sp.rowptr[pos]; b < sp.rowptr[pos + 1]; ++b) row_of[b] = pos;
  std::vector<std::vector<i64>> colblk(ncl);  // per elimination position: blocks (k, i), k before i
  for (i64 pos : f.rows)
    for (i64 b = sp.rowptr[pos] + 1; b < sp.rowptr[pos + 1]; ++b) colblk[sp.epos[sp.colidx[b]]].push_back(b);
  struct Rec {
    i64 target, src, blk;
  };
  auto by_target = [](const Rec& a, const Rec& b) {
    return a.target < b.target || (a.target == b.target && a.src < b.src);
  };
  p->fwd.resize(f.nflev);
  p->bwd.resize(f.nblev);
  // A target whose sources add up to more than 1.5 kt rows of K is cut at
  // segment boundaries into parts of about kt: the target's chain is the
  // level's critical path.  Part 0 subtracts its sum from the target; the
  // others store theirs in the partial buffer, and a reduction subtracts
  // them in part order (deterministic).
  const i64 kt = tune_knob("solve.split_k", 2048);
  std::vector<std::vector<Rec>> frec(f.nflev), brec(f.nblev);
  std::vector<i64> fneed(f.nflev, 0), bneed(f.nblev, 0);
  auto parts_of = [&](i64 ksum) -> i64 { return ksum * 2 > 3 * kt ? (ksum + kt - 1) / kt : 1; };
  auto need_of = [&](const std::vector<Rec>& recs) {
    i64 need = 0;
    for (size_t r = 0; r < recs.size();) {
      const i64 ct = sp.eorder[recs[r].target];
      i64 ksum = 0;
      for (; r < recs.size() && sp.eorder[recs[r].target] == ct; ++r)
        ksum += mb[sp.eorder[recs[r].src]];
      need += (parts_of(ksum) - 1) * nrhs * mb[ct];
    }
    return need;
  };
#pragma omp parallel for schedule(dynamic, 1)
  for (int lv = 0; lv < f.nflev; ++lv) {
    std::vector<Rec>& recs = frec[lv];
    for (i64 pk : fl[lv])
      for (i64 b = sp.rowptr[pk] + 1; b < sp.rowptr[pk + 1]; ++b) recs.push_back({sp.epos[sp.colidx[b]], pk, b});
    std::sort(recs.begin(), recs.end(), by_target);
    fneed[lv] = need_of(recs);
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int lv = 0; lv < f.nblev; ++lv) {
    std::vector<Rec>& recs = brec[lv];
    for (i64 pj : bl[lv])
      for (i64 b : colblk[pj]) recs.push_back({row_of[b], pj, b});
    std::sort(recs.begin(), recs.end(), by_target);
    bneed[lv] = need_of(recs);
  }
  i64 pcap = 1;
  for (i64 v : fneed) pcap = std::max(pcap, v);
  for (i64 v : bneed) pcap = std::max(pcap, v);
  T* part;
  if (arena) {
    part = static_cast<T*>(arena->take(sizeof(T) * pcap));
  } else {
    p->part.reset(sizeof(T) * pcap);
    part = p->part.as<T>();
  }
  p->part_ptr = part;
  p->y_ptr = y;
  p->w_ptr = w;
  std::vector<std::vector<SchurReduce>> fred(f.nflev), bred(f.nblev);
  // one level's items: sources of each target in elimination order, cut into parts
  auto build_level = [&](const std::vector<Rec>& recs, GemmBatch& g, std::vector<SchurReduce>& reds, T* vec,
                         bool fwd_side) {
    g.mode = GEMM_SUB;
    i64 poff = 0;
    for (size_t r = 0; r < recs.size();) {
      const i64 ct = sp.eorder[recs[r].target];
      size_t e = r;
      i64 ksum = 0;
      for (; e < recs.size() && sp.eorder[recs[e].target] == ct; ++e) ksum += mb[sp.eorder[recs[e].src]];
      const i64 np = parts_of(ksum);
      const i64 len = nrhs * mb[ct];
      i64 acc = 0, part_no = 0;
      GemmItem* it = nullptr;
      for (size_t q = r; q < e; ++q) {
        if (!it) {
          it = &g.item(N, int(mb[ct]), N, int(mb[ct]));
          if (part_no == 0) {
            GemmBatch::set_out(*it, 0, vec + sp.soff[ct] * nrhs, nrhs, false);
          } else {
            GemmBatch::set_out(*it, 0, part + poff + (part_no - 1) * len, nrhs, false);
            it->store = 1;
          }
        }
        const i64 cs = sp.eorder[recs[q].src];
        if (fwd_side) {
          // u_i^T -= u_k^T Z_ki  (Z_ki: m_k x m_i, ld m_k)
          g.seg(y + sp.soff[cs] * nrhs, N, false, S + sp.blk_off[recs[q].blk], int(mb[cs]), false, int(mb[cs]));
        } else {
          // x_k^T -= x_j^T Z_kj^T  (Z_kj: m_k x m_j, ld m_k; its transpose m_j x m_k, ld m_j)
          if (ST)
            g.seg(w + sp.soff[cs] * nrhs, N, false, ST + sp.blk_off[recs[q].blk], int(mb[cs]), false, int(mb[cs]));
          else
            g.seg(w + sp.soff[cs] * nrhs, N, false, S + sp.blk_off[recs[q].blk], int(mb[ct]), true, int(mb[cs]));
        }
        acc += mb[cs];
        if (part_no < np - 1 && acc * np >= (part_no + 1) * ksum) {
          ++part_no;
          it = nullptr;
        }
      }
      if (np > 1) {
        reds.push_back({sp.soff[ct] * nrhs, poff, int32_t(len), int32_t(np - 1)});
        poff += (np - 1) * len;
      }
      r = e;
    }
  };
#pragma omp parallel for schedule(dynamic, 1)
  for (int lv = 0; lv < f.nflev; ++lv) {
    build_level(frec[lv], p->fwd[lv], fred[lv], y, true);
    std::vector<Rec>().swap(frec[lv]);
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int lv = 0; lv < f.nblev; ++lv) {
    build_level(brec[lv], p->bwd[lv], bred[lv], w, false);
    std::vector<Rec>().swap(brec[lv]);
  }
  std::vector<SchurReduce> reds;
  p->fred_off.assign(f.nflev, 0);
  p->fred_cnt.assign(f.nflev, 0);
  p->bred_off.assign(f.nblev, 0);
  p->bred_cnt.assign(f.nblev, 0);
  for (int lv = 0; lv < f.nflev; ++lv) {
    p->fred_off[lv] = int(reds.size());
    p->fred_cnt[lv] = int(fred[lv].size());
    reds.insert(reds.end(), fred[lv].begin(), fred[lv].end());
  }
  for (int lv = 0; lv < f.nblev; ++lv) {
    p->bred_off[lv] = int(reds.size());
    p->bred_cnt[lv] = int(bred[lv].size());
    reds.insert(reds.end(), bred[lv].begin(), bred[lv].end());
  }
  if (!reds.empty()) {
    const size_t bytes = reds.size() * sizeof(SchurReduce);
    void* dst;
    if (arena) {
      dst = arena->take(bytes);
    } else {
      p->red.reset(bytes);
      dst = p->red.ptr;
    }
    HIPCHECK(hipMemcpyAsync(dst, reds.data(), bytes, hipMemcpyHostToDevice, current_stream()));
    HIPCHECK(hipStreamSynchronize(current_stream()));
    p->d_red = static_cast<const SchurReduce*>(dst);
  }
  // v_i^T = u_i^T D_i^{-1}: D_i^{-1} is symmetric (D_i is), read as stored
  for (i64 pos : f.rows) {
    const i64 c = sp.eorder[pos];
    GemmItem& it = p->diag.item(N, int(mb[c]), N, int(mb[c]));
    GemmBatch::set_out(it, 0, w + sp.soff[c] * nrhs, nrhs, false);
    p->diag.seg(y + sp.soff[c] * nrhs, N, false, Inv + f.inv_off[pos], int(mb[c]), false, int(mb[c]));
  }
  // V sweep: z_t^T = [z_t^b; y_t]^T Q_t^T, per level from the root
  p->down.resize(L + 1);
  for (int k = L; k >= 0; --k) {
    for (i64 c = tr.first_at_level(k); c < tr.first_at_level(k) + tr.count_at_level(k); ++c) {
      if (na[c] == 0) continue;
      GemmItem& it = p->down[k].item(N, int(na[c]), N, int(na[c]));
      GemmBatch::set_out(it, 0, zslot(c), nrhs, false);
      if (kp[c] > 0)
        p->down[k].seg(zslot((c - 1) / 2) + son_off(c) * nrhs, N, false, Q + sp.q_off[c], int(na[c]), true,
                       int(kp[c]));
      if (mb[c] > 0)
        p->down[k].seg(w + sp.soff[c] * nrhs, N, false, Q + sp.q_off[c] + kp[c] * na[c], int(na[c]), true,
                       int(mb[c]));
    }
  }
  std::vector<GemmBatch*> all;
  for (auto& g : p->up) all.push_back(&g);
  for (auto& g : p->down) all.push_back(&g);
  for (auto& g : p->fwd) all.push_back(&g);
  for (auto& g : p->bwd) all.push_back(&g);
  all.push_back(&p->diag);
  for (GemmBatch* g : all) {
    g->role = ROLE_SOLVE;
    g->prec = sizeof(T) == 4 ? 1 : 0;
  }
  HIPCHECK(hipStreamSynchronize(current_stream()));
  if (arena) upload_batches_into(all, *arena, current_stream());
  else upload_batches(all, p->desc);
  return p;
}

// zin (tree order, T) holds the right-hand side; on return zin holds
// V (L D L^T)^{-1} U^T zin in tree order.
template <class T>
static void apply_tree(h2_factor& f, SolvePlan& p, hipStream_t st) {
  const int L = f.sp->H->tree.depth;
  auto record = [&](hipStream_t s) {
    for (int k = 0; k <= L; ++k) p.up[k].launch<T>(s);
    for (int lv = 0; lv < f.nflev; ++lv) {
      p.fwd[lv].launch<T>(s);
      if (p.fred_cnt[lv] > 0)
        launch_schur_reduce<T>(p.d_red + p.fred_off[lv], p.fred_cnt[lv], static_cast<const T*>(p.part_ptr),
                               static_cast<T*>(p.y_ptr), s);
    }
    p.diag.launch<T>(s);
    for (int lv = 0; lv < f.nblev; ++lv) {
      p.bwd[lv].launch<T>(s);
      if (p.bred_cnt[lv] > 0)
        launch_schur_reduce<T>(p.d_red + p.bred_off[lv], p.bred_cnt[lv], static_cast<const T*>(p.part_ptr),
                               static_cast<T*>(p.w_ptr), s);
    }
    for (int k = L; k >= 0; --k) p.down[k].launch<T>(s);
  };
  if (trace_level() >= 3) {
    // every sweep launch timed on its own (eager), summed by launch size
    struct Rec {
      const GemmBatch* b;
      hipEvent_t e0, e1;
    };
    std::vector<Rec> recs;
    auto timed = [&](const GemmBatch& b) {
      Rec r{&b, nullptr, nullptr};
      HIPCHECK(hipEventCreate(&r.e0));
      HIPCHECK(hipEventCreate(&r.e1));
      HIPCHECK(hipEventRecord(r.e0, st));
      b.launch<T>(st);
      HIPCHECK(hipEventRecord(r.e1, st));
      recs.push_back(r);
    };
    for (int k = 0; k <= L; ++k) timed(p.up[k]);
    for (int lv = 0; lv < f.nflev; ++lv) {
      timed(p.fwd[lv]);
      if (p.fred_cnt[lv] > 0)
        launch_schur_reduce<T>(p.d_red + p.fred_off[lv], p.fred_cnt[lv], static_cast<const T*>(p.part_ptr),
                               static_cast<T*>(p.y_ptr), st);
    }
    timed(p.diag);
    for (int lv = 0; lv < f.nblev; ++lv) {
      timed(p.bwd[lv]);
      if (p.bred_cnt[lv] > 0)
        launch_schur_reduce<T>(p.d_red + p.bred_off[lv], p.bred_cnt[lv], static_cast<const T*>(p.part_ptr),
                               static_cast<T*>(p.w_ptr), st);
    }
    for (int k = L; k >= 0; --k) timed(p.down[k]);
    HIPCHECK(hipStreamSynchronize(st));
    const int64_t edges[] = {0, 256, 1024, 4096, 16384, 65536, int64_t(1) << 40};
    double ms[6] = {0}, fl[6] = {0};
    int cnt[6] = {0};
    for (const Rec& r : recs) {
      float t = 0;
      HIPCHECK(hipEventElapsedTime(&t, r.e0, r.e1));
      int bkt = 0;
      while (bkt < 5 && r.b->ntiles >= edges[bkt + 1]) ++bkt;
      ms[bkt] += t;
      fl[bkt] += r.b->flops;
      ++cnt[bkt];
      (void)hipEventDestroy(r.e0);
      (void)hipEventDestroy(r.e1);
    }
    for (int bkt = 0; bkt < 6; ++bkt)
      if (cnt[bkt])
        std::fprintf(stderr, "[h2sp] solve sweep launches of %lld..%lld work-groups: %d launches, %.1f ms, %.2f TFLOP/s\n",
                     (long long)edges[bkt], (long long)edges[bkt + 1] - 1, cnt[bkt], ms[bkt],
                     fl[bkt] / (ms[bkt] * 1e-3) / 1e12);
    return;
  }
  if (p.eager) record(st);
  else p.apply.run(st, record);
}

SolvePlan& solve_plan(h2_factor& f, i64 nrhs) {
  if (!f.solve || f.solve->nrhs != nrhs || f.solve->tune_gen != tune_generation()) {
    f.solve.reset();
    if (f.sp->precision == H2_MIXED) f.solve = make_solve_plan<float>(f, nrhs);
    else f.solve = make_solve_plan<double>(f, nrhs);
  }
  return *f.solve;
}

// acc += V (LDL^T)^{-1} U^T r: r, acc in tree order, FP64, RHS-fastest; in
// mixed precision r is scaled column by column to unit norm for the FP32
// application and scaled back into acc
static void correction(h2_factor& f, SolvePlan& p, const double* r_tree, double* acc, const double* colscale_dev,
                       hipStream_t st) {
  const i64 n = f.sp->H->tree.n, nrhs = p.nrhs;
  if (f.sp->precision == H2_MIXED) {
    launch_scale_to_f_rm(r_tree, colscale_dev, static_cast<float*>(p.zin_ptr), n, nrhs, st);
    apply_tree<float>(f, p, st);
    launch_add_scaled_f_rm(static_cast<const float*>(p.zin_ptr), colscale_dev, acc, n, nrhs, st);
  } else {
    HIPCHECK(hipMemcpyAsync(p.zin_ptr, r_tree, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, st));
    apply_tree<double>(f, p, st);
    launch_add(static_cast<const double*>(p.zin_ptr), acc, n * nrhs, n * nrhs, 1, st);
  }
}

}  // namespace h2

using namespace h2;

// One preconditioner application in original order: x = V (LDL^T)^{-1} U^T b.
int apply_inverse_impl(h2_factor* f, const double* b, double* x, i64 nrhs, i64 ld) {
  h2_matrix& H = *f->sp->H;
  const i64 n = H.tree.n;
  hipStream_t st = current_stream();
  SolvePlan& p = solve_plan(*f, nrhs);
  DeviceBuffer rt(sizeof(double) * n * nrhs), ones(sizeof(double) * nrhs);
  launch_fill(ones.as<double>(), nrhs, 1.0, st);
  launch_gather_rm(b, ld, H.d_perm.as<i64>(), rt.as<double>(), n, nrhs, st);
  launch_fill(p.rs_ptr, n * nrhs, 0.0, st);
  correction(*f, p, rt.as<double>(), p.rs_ptr, ones.as<double>(), st);
  launch_scatter_rm(p.rs_ptr, H.d_perm.as<i64>(), x, ld, n, nrhs, st);
  HIPCHECK(hipStreamSynchronize(st));
  return H2_OK;
}

// The same application without allocating device memory: every vector and
// the work lists of a plan made for this call live in the library's static
// scratch array (kNoAllocScratchBytes per GPU), launched eagerly.  The
// array is shared by every call on its GPU: calls that overlap race.
int apply_inverse_noalloc_impl(h2_factor* f, const double* b, double* x, i64 nrhs, i64 ld) {
  h2_matrix& H = *f->sp->H;
  const i64 n = H.tree.n;
  hipStream_t st = current_stream();
  void* base = nullptr;
  HIPCHECK(noalloc_scratch(&base));
  DeviceArena ar{static_cast<char*>(base), kNoAllocScratchBytes, 0, "h2_apply_inverse_noalloc: the scratch array"};
  double* rt = static_cast<double*>(ar.take(sizeof(double) * n * nrhs));
  double* ones = static_cast<double*>(ar.take(sizeof(double) * nrhs));
  std::unique_ptr<SolvePlan> p = f->sp->precision == H2_MIXED ? make_solve_plan<float>(*f, nrhs, &ar)
                                                               : make_solve_plan<double>(*f, nrhs, &ar);
  launch_fill(ones, nrhs, 1.0, st);
  launch_gather_rm(b, ld, H.d_perm.as<i64>(), rt, n, nrhs, st);
  launch_fill(p->rs_ptr, n * nrhs, 0.0, st);
  correction(*f, *p, rt, p->rs_ptr, ones, st);
  launch_scatter_rm(p->rs_ptr, H.d_perm.as<i64>(), x, ld, n, nrhs, st);
  HIPCHECK(hipStreamSynchronize(st));
  return H2_OK;
}

namespace h2 {

// State of a solve: right-hand side, solution and residual in tree order,
// RHS-fastest, FP64; the matvec plan of the operator A and the solve plan of
// the factor.
struct SolveState {
  h2_factor& f;
  const h2_matrix& A;
  SolvePlan& p;
  MatvecPlan& mv;
  MatvecPlanView mvb;
  i64 n, nrhs;
  hipStream_t st;
  double* bt;     // b
  double* xt;     // x
  double* rt;     // b - A x
  double* nrm;    // 2 nrhs: ||r_j||^2, ||b_j||^2
  double* part;   // scratch of the reductions
  std::vector<double> bnorm;
  std::vector<hipEvent_t> ev;  // pairs of (start, end) events: precond, matvec
  std::vector<int> ev_kind;    // 0: preconditioner, 1: matvec
  void mark_begin() {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    HIPCHECK(hipEventRecord(e, st));
    ev.push_back(e);
  }
  void mark_end(int kind) {
    mark_begin();
    ev_kind.push_back(kind);
  }
  // y = A x_in (x_in in tree order, RHS-fastest) into the matvec plan's yt
  void matvec(const double* x_in) {
    mark_begin();
    HIPCHECK(hipMemcpyAsync(mvb.xt, x_in, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, st));
    run_matvec_tree(A, mv, st);
    mark_end(1);
  }
  // r = b - A x and its column norms; returns max_j ||r_j|| / ||b_j||
  double residual(std::vector<double>& h_nrm) {
    matvec(xt);
    launch_residual_rm(bt, mvb.yt, rt, n, nrhs, part, nrm, st);
    HIPCHECK(hipMemcpyAsync(h_nrm.data(), nrm, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    double res = 0;
    for (i64 j = 0; j < nrhs; ++j) {
      const double q = bnorm[j] > 0 ? std::sqrt(h_nrm[j]) / bnorm[j] : 0.0;
      if (!std::isfinite(q)) return q;
      res = std::max(res, q);
    }
    return res;
  }
};

// Flexible GMRES (Saad 1993), right preconditioned by M^{-1} (the factor of S
// inside U^T and V), restarted every `m` steps, many right-hand sides at once
// (one Krylov space per column; the columns share every launch).  Arnoldi by
// classical Gram-Schmidt applied twice, with the Hessenberg columns on the
// host, reduced by Givens rotations per right-hand side.  Starts from the
// state's x and r (r = b - A x, column norms in h_nrm); stops when the true
// residual is at or below tol or after `budget` steps.  Returns the steps
// taken; res holds the final residual.
static int fgmres(SolveState& S, int m, int budget, double tol, std::vector<double>& h_nrm, double& res) {
  const i64 n = S.n, nrhs = S.nrhs, len = n * nrhs;
  hipStream_t st = S.st;
  DeviceBuffer vb(sizeof(double) * size_t(m + 1) * len), zb(sizeof(double) * size_t(m) * len),
      w(sizeof(double) * len), c1(sizeof(double) * (m + 1) * nrhs), c2(sizeof(double) * (m + 1) * nrhs),
      yd(sizeof(double) * m * nrhs), cs(sizeof(double) * nrhs), part(sizeof(double) * size_t(m + 1) * nrhs *
                                                                      residual_rm_blocks(n));
  double* V = vb.as<double>();
  double* Z = zb.as<double>();
  std::vector<double> ones(nrhs, 1.0);
  HIPCHECK(hipMemcpyAsync(cs.ptr, ones.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
  // per column: Hessenberg (m + 1) x m column-major, rotations, right-hand side g
  std::vector<double> H(size_t(nrhs) * (m + 1) * m), gc(size_t(nrhs) * m), gs(size_t(nrhs) * m),
      g(size_t(nrhs) * (m + 1)), h1((m + 1) * nrhs), h2((m + 1) * nrhs), nw(nrhs), y(size_t(m) * nrhs);
  int steps = 0;
  while (steps < budget) {
    // v_0 = r / ||r||, g = ||r|| e_1
    HIPCHECK(hipMemcpyAsync(S.nrm, h_nrm.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    launch_scale_cols(S.rt, S.nrm, V, n, nrhs, st);
    std::fill(g.begin(), g.end(), 0.0);
    for (i64 c = 0; c < nrhs; ++c) g[c * (m + 1)] = std::sqrt(h_nrm[c]);
    int j = 0;
    for (; j < m && steps < budget; ++j, ++steps) {
      double* vj = V + j * len;
      double* zj = Z + j * len;
      // z_j = M^{-1} v_j (columns of unit norm: no scaling), w = A z_j
      S.mark_begin();
      launch_fill(zj, len, 0.0, st);
      correction(S.f, S.p, vj, zj, cs.as<double>(), st);
      S.mark_end(0);
      S.matvec(zj);
      HIPCHECK(hipMemcpyAsync(w.ptr, S.mvb.yt, sizeof(double) * len, hipMemcpyDeviceToDevice, st));
      // two passes of classical Gram-Schmidt against v_0 .. v_j, then ||w||
      launch_multi_dot(V, len, j + 1, w.as<double>(), n, nrhs, part.as<double>(), c1.as<double>(), st);
      launch_multi_axpy(V, len, j + 1, c1.as<double>(), -1.0, w.as<double>(), n, nrhs, st);
      launch_multi_dot(V, len, j + 1, w.as<double>(), n, nrhs, part.as<double>(), c2.as<double>(), st);
      launch_multi_axpy(V, len, j + 1, c2.as<double>(), -1.0, w.as<double>(), n, nrhs, st);
      launch_multi_dot(w.as<double>(), 0, 1, w.as<double>(), n, nrhs, part.as<double>(), S.nrm, st);
      launch_scale_cols(w.as<double>(), S.nrm, V + (j + 1) * len, n, nrhs, st);
      HIPCHECK(hipMemcpyAsync(h1.data(), c1.ptr, sizeof(double) * (j + 1) * nrhs, hipMemcpyDeviceToHost, st));
      HIPCHECK(hipMemcpyAsync(h2.data(), c2.ptr, sizeof(double) * (j + 1) * nrhs, hipMemcpyDeviceToHost, st));
      HIPCHECK(hipMemcpyAsync(nw.data(), S.nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      double est = 0;
      for (i64 c = 0; c < nrhs; ++c) {
        double* hc = &H[size_t(c) * (m + 1) * m + size_t(j) * (m + 1)];
        for (int i = 0; i <= j; ++i) hc[i] = h1[i * nrhs + c] + h2[i * nrhs + c];
        hc[j + 1] = std::sqrt(nw[c]);
        double* gcc = &gc[size_t(c) * m];
        double* gss = &gs[size_t(c) * m];
        for (int i = 0; i < j; ++i) {
          const double a = hc[i], b = hc[i + 1];
          hc[i] = gcc[i] * a + gss[i] * b;
          hc[i + 1] = -gss[i] * a + gcc[i] * b;
        }
        const double a = hc[j], b = hc[j + 1], r = std::hypot(a, b);
        gcc[j] = r > 0 ? a / r : 1.0;
        gss[j] = r > 0 ? b / r : 0.0;
        hc[j] = r;
        hc[j + 1] = 0.0;
        double* gg = &g[size_t(c) * (m + 1)];
        gg[j + 1] = -gss[j] * gg[j];
        gg[j] = gcc[j] * gg[j];
        if (S.bnorm[c] > 0) est = std::max(est, std::abs(gg[j + 1]) / S.bnorm[c]);
      }
      if (!std::isfinite(est)) {
        ++steps;
        ++j;
        break;
      }
      if (est <= 0.5 * tol) {
        ++steps;
        ++j;
        break;
      }
    }
    // x += Z y, y from the triangular system of each column
    for (i64 c = 0; c < nrhs; ++c) {
      const double* hc = &H[size_t(c) * (m + 1) * m];
      const double* gg = &g[size_t(c) * (m + 1)];
      for (int i = j - 1; i >= 0; --i) {
        double acc = gg[i];
        for (int k = i + 1; k < j; ++k) acc -= hc[size_t(k) * (m + 1) + i] * y[k * nrhs + c];
        const double d = hc[size_t(i) * (m + 1) + i];
        y[i * nrhs + c] = d != 0.0 ? acc / d : 0.0;
      }
    }
    HIPCHECK(hipMemcpyAsync(yd.ptr, y.data(), sizeof(double) * j * nrhs, hipMemcpyHostToDevice, st));
    launch_multi_axpy(Z, len, j, yd.as<double>(), 1.0, S.xt, n, nrhs, st);
    res = S.residual(h_nrm);
    if (!(res > tol)) break;  // converged (or not finite)
  }
  return steps;
}

}  // namespace h2

// Solve of A x = b with the factor f as approximate inverse (its matrix's
// tree); x in tree order (p.rs), r = b - A x.
static int solve_impl2(h2_factor* f, const h2_matrix& A, const double* b, double* x, i64 nrhs, i64 ld,
                       const h2_solve_opts* o, h2_solve_info* info) {
  const i64 n = A.tree.n;
  hipStream_t st = current_stream();
  const auto t_plan0 = std::chrono::steady_clock::now();
  SolvePlan& p = solve_plan(*f, nrhs);
  MatvecPlan& mv = matvec_plan(A, nrhs);
  const double plan_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_plan0).count();
  const double tol = o ? o->tol : 1e-10;
  const int max_iter = o ? std::max(1, o->max_iter) : 30;
  const int method = o ? o->method : H2_SOLVE_AUTO;
  int restart = o && o->restart > 0 ? o->restart : 30;
  if (method < H2_SOLVE_AUTO || method > H2_SOLVE_GMRES) fail(H2_EINVAL, "unknown solve method");
  if (restart > 64) fail(H2_EINVAL, "GMRES restart above 64");
  const size_t vec = sizeof(double) * n * nrhs;
  DeviceBuffer bt(vec), rt(vec), xprev(method == H2_SOLVE_AUTO ? vec : 0), nrm(sizeof(double) * 2 * nrhs),
      cs(sizeof(double) * nrhs), part(sizeof(double) * 2 * nrhs * residual_rm_blocks(n));
  SolveState S{*f, A, p, mv, matvec_buffers(mv), n, nrhs, st, bt.as<double>(), p.rs_ptr,
               rt.as<double>(), nrm.as<double>(), part.as<double>(), {}, {}, {}};
  launch_gather_rm(b, ld, A.d_perm.as<i64>(), S.bt, n, nrhs, st);
  launch_fill(S.xt, n * nrhs, 0.0, st);
  std::vector<double> h_nrm(2 * nrhs), h_cs(nrhs);
  // r = b (x = 0) and the column norms of b
  launch_fill(S.mvb.yt, n * nrhs, 0.0, st);
  launch_residual_rm(S.bt, S.mvb.yt, S.rt, n, nrhs, S.part, S.nrm, st);
  HIPCHECK(hipMemcpyAsync(h_nrm.data(), S.nrm, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  S.bnorm.resize(nrhs);
  for (i64 j = 0; j < nrhs; ++j) S.bnorm[j] = std::sqrt(h_nrm[nrhs + j]);
  double res = 0;
  for (i64 j = 0; j < nrhs; ++j) res = std::max(res, S.bnorm[j] > 0 ? 1.0 : 0.0);
  int refine = 0, gm = 0, stall = 0;
  bool to_gmres = method == H2_SOLVE_GMRES;
  double prev = res;
  while (!to_gmres && refine < max_iter && res > tol) {
    for (i64 j = 0; j < nrhs; ++j) {
      const double rn = std::sqrt(h_nrm[j]);
      h_cs[j] = rn > 0 ? rn : 1.0;
    }
    if (method == H2_SOLVE_AUTO) HIPCHECK(hipMemcpyAsync(xprev.ptr, S.xt, vec, hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipMemcpyAsync(cs.ptr, h_cs.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    S.mark_begin();
    correction(*f, p, S.rt, S.xt, cs.as<double>(), st);
    S.mark_end(0);
    ++refine;
    res = S.residual(h_nrm);
    if (method != H2_SOLVE_AUTO) {
      if (!std::isfinite(res)) break;
      continue;
    }
    const double ratio = res / prev;
    if (!std::isfinite(res) || ratio > 2.0) {
      // diverging: back to the previous x (and its residual), then GMRES
      HIPCHECK(hipMemcpyAsync(S.xt, xprev.ptr, vec, hipMemcpyDeviceToDevice, st));
      res = S.residual(h_nrm);
      to_gmres = true;
      break;
    }
    stall = ratio > 0.9 ? stall + 1 : 0;
    prev = res;
    if (stall >= 3) to_gmres = true;
  }
  if (to_gmres && res > tol && refine < max_iter && std::isfinite(res))
    gm = fgmres(S, restart, max_iter - refine, tol, h_nrm, res);
  launch_scatter_rm(S.xt, A.d_perm.as<i64>(), x, ld, n, nrhs, st);
  HIPCHECK(hipStreamSynchronize(st));
  double t_prec = 0, t_mv = 0;
  for (size_t e = 0; e < S.ev_kind.size(); ++e) {
    float a = 0;
    HIPCHECK(hipEventElapsedTime(&a, S.ev[2 * e], S.ev[2 * e + 1]));
    (S.ev_kind[e] == 0 ? t_prec : t_mv) += a * 1e-3;
  }
  for (auto e : S.ev) (void)hipEventDestroy(e);
  if (info) {
    info->iters = refine + gm;
    info->max_rel_residual = res;
    info->seconds[0] = t_prec;
    info->seconds[1] = t_mv;
    info->seconds[2] = plan_s;
    info->gmres_steps = gm;
    info->refine_steps = refine;
  }
  if (!(res <= tol)) return H2_ENOCONV;
  return H2_OK;
}

int solve_impl(h2_factor* f, const double* b, double* x, i64 nrhs, i64 ld, const h2_solve_opts* o,
               h2_solve_info* info) {
  return solve_impl2(f, *f->sp->H, b, x, nrhs, ld, o, info);
}

// Solve with another matrix of the same points as the operator (the factor of
// a coarser H^2 matrix as preconditioner of a finer one, Section 5.5).
int solve_with_impl(const h2_matrix* A, h2_factor* f, const double* b, double* x, i64 nrhs, i64 ld,
                    const h2_solve_opts* o, h2_solve_info* info) {
  const h2_matrix& B = *f->sp->H;
  if (A->tree.n != B.tree.n || A->tree.perm != B.tree.perm || A->tree.depth != B.tree.depth)
    fail(H2_EINVAL, "the operator and the factor's matrix must share points and cluster tree");
  const_cast<h2_matrix*>(A)->upload_all();
  return solve_impl2(f, *A, b, x, nrhs, ld, o, info);
}

h2_factor::~h2_factor() = default;
