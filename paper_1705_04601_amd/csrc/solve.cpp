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

template <class T>
static std::unique_ptr<SolvePlan> make_solve_plan(h2_factor& f, i64 nrhs) {
  TraceTimer tt("solve-plan");
  h2_sparse& sp = *f.sp;
  h2_matrix& H = *sp.H;
  const Tree& tr = H.tree;
  const i64 n = tr.n, ncl = sp.ncl;
  const int L = tr.depth;
  auto p = std::make_unique<SolvePlan>();
  p->nrhs = nrhs;
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
  p->zin.reset(sizeof(T) * n * nrhs);       // right-hand side in tree order (leaf z)
  p->zbuf.reset(sizeof(T) * std::max<i64>(zs, 1));
  p->y.reset(sizeof(T) * n * nrhs);
  p->w.reset(sizeof(T) * n * nrhs);
  p->rs.reset(sizeof(double) * n * nrhs);
  p->colscale.reset(sizeof(double) * nrhs);
  T* zin = p->zin.as<T>();
  T* zb = p->zbuf.as<T>();
  T* y = p->y.as<T>();
  T* w = p->w.as<T>();
  const T* Q = (sp.precision == H2_MIXED) ? sp.dQt.as<T>() : reinterpret_cast<const T*>(sp.dQ.as<double>());
  const T* S = sp.dS.as<T>();
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
#pragma omp parallel for schedule(dynamic, 1)
  for (int lv = 0; lv < f.nflev; ++lv) {
    std::vector<Rec> recs;
    for (i64 pk : fl[lv])
      for (i64 b = sp.rowptr[pk] + 1; b < sp.rowptr[pk + 1]; ++b) recs.push_back({sp.epos[sp.colidx[b]], pk, b});
    std::sort(recs.begin(), recs.end(), by_target);
    GemmBatch& g = p->fwd[lv];
    g.mode = GEMM_SUB;
    for (size_t r = 0; r < recs.size();) {
      const i64 ci = sp.eorder[recs[r].target];
      // u_i^T -= u_k^T Z_ki  (Z_ki: m_k x m_i, ld m_k)
      GemmItem& it = g.item(N, int(mb[ci]), N, int(mb[ci]));
      GemmBatch::set_out(it, 0, y + sp.soff[ci] * nrhs, nrhs, false);
      for (; r < recs.size() && sp.eorder[recs[r].target] == ci; ++r) {
        const i64 ck = sp.eorder[recs[r].src];
        g.seg(y + sp.soff[ck] * nrhs, N, false, S + sp.blk_off[recs[r].blk], int(mb[ck]), false, int(mb[ck]));
      }
    }
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int lv = 0; lv < f.nblev; ++lv) {
    std::vector<Rec> recs;
    for (i64 pj : bl[lv])
      for (i64 b : colblk[pj]) recs.push_back({row_of[b], pj, b});
    std::sort(recs.begin(), recs.end(), by_target);
    GemmBatch& g = p->bwd[lv];
    g.mode = GEMM_SUB;
    for (size_t r = 0; r < recs.size();) {
      const i64 ck = sp.eorder[recs[r].target];
      // x_k^T -= x_j^T Z_kj^T  (Z_kj: m_k x m_j, ld m_k)
      GemmItem& it = g.item(N, int(mb[ck]), N, int(mb[ck]));
      GemmBatch::set_out(it, 0, w + sp.soff[ck] * nrhs, nrhs, false);
      for (; r < recs.size() && sp.eorder[recs[r].target] == ck; ++r) {
        const i64 cj = sp.eorder[recs[r].src];
        g.seg(w + sp.soff[cj] * nrhs, N, false, S + sp.blk_off[recs[r].blk], int(mb[ck]), true, int(mb[cj]));
      }
    }
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
  for (GemmBatch* g : all) g->role = ROLE_SOLVE;
  HIPCHECK(hipStreamSynchronize(current_stream()));
  upload_batches(all, p->desc);
  return p;
}

// zin (tree order, T) holds the right-hand side; on return zin holds
// V (L D L^T)^{-1} U^T zin in tree order.
template <class T>
static void apply_tree(h2_factor& f, SolvePlan& p, hipStream_t st) {
  const int L = f.sp->H->tree.depth;
  p.apply.run(st, [&](hipStream_t s) {
    for (int k = 0; k <= L; ++k) p.up[k].launch<T>(s);
    for (int lv = 0; lv < f.nflev; ++lv) p.fwd[lv].launch<T>(s);
    p.diag.launch<T>(s);
    for (int lv = 0; lv < f.nblev; ++lv) p.bwd[lv].launch<T>(s);
    for (int k = L; k >= 0; --k) p.down[k].launch<T>(s);
  });
}

SolvePlan& solve_plan(h2_factor& f, i64 nrhs) {
  if (!f.solve || f.solve->nrhs != nrhs) {
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
    launch_scale_to_f_rm(r_tree, colscale_dev, p.zin.as<float>(), n, nrhs, st);
    apply_tree<float>(f, p, st);
    launch_add_scaled_f_rm(p.zin.as<float>(), colscale_dev, acc, n, nrhs, st);
  } else {
    HIPCHECK(hipMemcpyAsync(p.zin.ptr, r_tree, sizeof(double) * n * nrhs, hipMemcpyDeviceToDevice, st));
    apply_tree<double>(f, p, st);
    launch_add(p.zin.as<double>(), acc, n * nrhs, n * nrhs, 1, st);
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
  launch_fill(p.rs.as<double>(), n * nrhs, 0.0, st);
  correction(*f, p, rt.as<double>(), p.rs.as<double>(), ones.as<double>(), st);
  launch_scatter_rm(p.rs.as<double>(), H.d_perm.as<i64>(), x, ld, n, nrhs, st);
  HIPCHECK(hipStreamSynchronize(st));
  return H2_OK;
}

// Iterative refinement.  x accumulates in tree order (p.rs), r = b - A_H2 x.
int solve_impl(h2_factor* f, const double* b, double* x, i64 nrhs, i64 ld, const h2_solve_opts* o,
               h2_solve_info* info) {
  h2_matrix& H = *f->sp->H;
  const i64 n = H.tree.n;
  hipStream_t st = current_stream();
  const auto t_plan0 = std::chrono::steady_clock::now();
  SolvePlan& p = solve_plan(*f, nrhs);
  MatvecPlan& mv = matvec_plan(H, nrhs);
  const double plan_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_plan0).count();
  // device time of the preconditioner applications and of the matvecs
  std::vector<hipEvent_t> ev;
  auto mark = [&]() {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    HIPCHECK(hipEventRecord(e, st));
    ev.push_back(e);
  };
  MatvecPlanView mvb = matvec_buffers(mv);
  const size_t vec = sizeof(double) * n * nrhs;
  DeviceBuffer bt(vec), rt(vec), nrm(sizeof(double) * 2 * nrhs), cs(sizeof(double) * nrhs),
      part(sizeof(double) * 2 * nrhs * residual_rm_blocks(n));
  launch_gather_rm(b, ld, H.d_perm.as<i64>(), bt.as<double>(), n, nrhs, st);
  launch_fill(p.rs.as<double>(), n * nrhs, 0.0, st);
  std::vector<double> h_nrm(2 * nrhs), h_cs(nrhs);
  // r = b (x = 0) and the column norms of b for the first scaling
  launch_fill(mvb.yt, n * nrhs, 0.0, st);
  launch_residual_rm(bt.as<double>(), mvb.yt, rt.as<double>(), n, nrhs, part.as<double>(), nrm.as<double>(), st);
  HIPCHECK(hipMemcpyAsync(h_nrm.data(), nrm.ptr, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  std::vector<double> bnorm(nrhs);
  for (i64 j = 0; j < nrhs; ++j) bnorm[j] = std::sqrt(h_nrm[nrhs + j]);
  const double tol = o ? o->tol : 1e-10;
  const int max_iter = o ? std::max(1, o->max_iter) : 30;
  double res = 0;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    for (i64 j = 0; j < nrhs; ++j) {
      const double rn = std::sqrt(h_nrm[j]);
      h_cs[j] = rn > 0 ? rn : 1.0;
    }
    HIPCHECK(hipMemcpyAsync(cs.ptr, h_cs.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
    mark();
    correction(*f, p, rt.as<double>(), p.rs.as<double>(), cs.as<double>(), st);
    mark();
    // r = b - A x  (x = p.rs in tree order)
    HIPCHECK(hipMemcpyAsync(mvb.xt, p.rs.ptr, vec, hipMemcpyDeviceToDevice, st));
    run_matvec_tree(H, mv, st);
    mark();
    launch_residual_rm(bt.as<double>(), mvb.yt, rt.as<double>(), n, nrhs, part.as<double>(), nrm.as<double>(), st);
    HIPCHECK(hipMemcpyAsync(h_nrm.data(), nrm.ptr, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    res = 0;
    for (i64 j = 0; j < nrhs; ++j)
      res = std::max(res, bnorm[j] > 0 ? std::sqrt(h_nrm[j]) / bnorm[j] : 0.0);
    if (!std::isfinite(res)) break;
    if (res <= tol) break;
  }
  if (it > max_iter) it = max_iter;
  launch_scatter_rm(p.rs.as<double>(), H.d_perm.as<i64>(), x, ld, n, nrhs, st);
  HIPCHECK(hipStreamSynchronize(st));
  double t_prec = 0, t_mv = 0;
  for (size_t e = 0; e + 2 < ev.size(); e += 3) {
    float a = 0, c = 0;
    HIPCHECK(hipEventElapsedTime(&a, ev[e], ev[e + 1]));
    HIPCHECK(hipEventElapsedTime(&c, ev[e + 1], ev[e + 2]));
    t_prec += a * 1e-3;
    t_mv += c * 1e-3;
  }
  for (auto e : ev) (void)hipEventDestroy(e);
  if (info) {
    info->iters = it;
    info->max_rel_residual = res;
    info->seconds[0] = t_prec;
    info->seconds[1] = t_mv;
    info->seconds[2] = plan_s;
  }
  if (!(res <= tol)) return H2_ENOCONV;
  return H2_OK;
}

h2_factor::~h2_factor() = default;
