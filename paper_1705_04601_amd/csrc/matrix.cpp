// h2_matrix: construction, import, export and the FP64 H^2 matrix-vector
// product (Definition 4.9, the H^2 matrix): close part from kernel blocks kept on the device
// (or evaluated on the fly from the points when they do not fit), far part by
// the nested bases (upward pass, couplings, downward pass).
#include <cmath>
#include <cstdlib>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "batch.h"
#include "h2_internal.h"

namespace h2 {
void fill_structure(h2_matrix& H, const double* pts, i64 n, int dim, const h2_kernel& kern,
                    const h2_build_opts& o);
void build_chebyshev(h2_matrix& H, double tol, int rank_cap);

static void validate(const double* pts, i64 n, int dim, const h2_kernel* kernel,
                     const h2_build_opts* o) {
  if (!pts || !kernel || !o) fail(H2_EINVAL, "null argument");
  if (n < 1) fail(H2_EINVAL, "n must be >= 1");
  if (dim != 2 && dim != 3) fail(H2_EINVAL, "dim must be 2 or 3");
  if (kernel->kind != H2_KERNEL_INVDIST && kernel->kind != H2_KERNEL_EXP && kernel->kind != H2_KERNEL_IFMM)
    fail(H2_EUNSUPPORTED, "unknown kernel kind");
  if (!std::isfinite(kernel->scale) || !std::isfinite(kernel->diag)) fail(H2_EINVAL, "kernel constants not finite");
  if (kernel->kind == H2_KERNEL_IFMM && !(kernel->param > 0.0 && std::isfinite(kernel->param)))
    fail(H2_EINVAL, "H2_KERNEL_IFMM needs a finite param d > 0");
  if (o->leaf < 2 || o->leaf > 128) fail(H2_EINVAL, "leaf must be in [2, 128]");
  if (o->cheb < 2 || o->cheb > 8) fail(H2_EINVAL, "cheb must be in [2, 8]");
  int P = 1;
  for (int a = 0; a < dim; ++a) P *= o->cheb;
  if (P > 64) fail(H2_EUNSUPPORTED, "cheb^dim must be <= 64");
  if (!(o->eta >= 0.0) || !std::isfinite(o->eta)) fail(H2_EINVAL, "eta must be >= 0");
  if (!(o->recompress_tol >= 0.0)) fail(H2_EINVAL, "recompress_tol must be >= 0");
  for (i64 i = 0; i < n * dim; ++i)
    if (!std::isfinite(pts[i])) fail(H2_EINVAL, "point coordinates must be finite");
}

// Duplicate points give a zero distance in the kernel; detected on the sorted
// leaves (equal points always share a leaf: the split order is total).
static void check_duplicates(const h2_matrix& H) {
  const Tree& tr = H.tree;
  const int dim = tr.dim;
  const i64 f = tr.first_at_level(0), cnt = tr.count_at_level(0);
  for (i64 c = f; c < f + cnt; ++c)
    for (i64 i = tr.start[c]; i < tr.start[c] + tr.size[c]; ++i)
      for (i64 j = i + 1; j < tr.start[c] + tr.size[c]; ++j) {
        bool same = true;
        for (int a = 0; a < dim && same; ++a) same = H.x_tree[i * dim + a] == H.x_tree[j * dim + a];
        if (same) fail(H2_EINVAL, "duplicate points");
      }
}

}  // namespace h2

using namespace h2;

// One thread at a time per matrix (the batched entry points reject a matrix
// that appears twice); marked done only once every copy is in place, so that
// a failed upload is retried rather than leaving null device pointers.
void h2_matrix::upload_all() {
  if (on_device) return;
  d_x = upload(x_tree);
  d_nodes = upload(nodes);
  d_proj = upload(proj);
  d_basis = upload(basis);
  d_transfer = upload(transfer);
  d_perm = upload(tree.perm);
  on_device = true;
}

// ---------------------------------------------------------------- matvec plan
namespace h2 {

struct MatvecPlan {
  i64 nrhs = 0;
  int64_t tune_gen = 0;          // tuning generation the lists were planned under
  DeviceBuffer xt, yt, xhat, xtil, ytil, yhat, desc;
  DeviceBuffer close_blocks;     // kernel blocks of the close part, when resident
  GemmBatch close;
  std::vector<GemmBatch> up;     // per level (0 = leaves)
  GemmBatch xproj, coup, yproj;
  std::vector<GemmBatch> down;   // per level, applied from the top
  GemmBatch leafout;
  LaunchGraph graph;             // the whole product, captured once
};

// Whether the close part's kernel blocks (FP64) are kept on the device: when
// they take at most a quarter of the free device memory (idle cached blocks
// count as free).  H2SP_CLOSE_RESIDENT=0 generates them inside every product.
static bool close_blocks_fit(size_t bytes) {
  if (const char* e = std::getenv("H2SP_CLOSE_RESIDENT"))
    if (e[0] == '0') return false;
  size_t free_b = 0, total_b = 0;
  HIPCHECK(hipMemGetInfo(&free_b, &total_b));
  return bytes <= (free_b + cached_device_bytes()) / 4;
}

static std::unique_ptr<MatvecPlan> make_matvec_plan(h2_matrix& H, i64 nrhs) {
  H.upload_all();
  auto mp = std::make_unique<MatvecPlan>();
  MatvecPlan& p = *mp;
  p.tune_gen = tune_generation();
  const Tree& tr = H.tree;
  const i64 n = tr.n, ncl = tr.ncl();
  const int dim = tr.dim, P = H.P, L = tr.depth;
  p.nrhs = nrhs;
  p.xt.reset(sizeof(double) * n * nrhs);
  p.yt.reset(sizeof(double) * n * nrhs);
  std::vector<i64> hoff(ncl, -1), poff(ncl, -1);
  i64 hs = 0, ps = 0;
  for (i64 c = 0; c < ncl; ++c)
    if (H.ff[c]) {
      hoff[c] = hs;
      hs += i64(H.rank[c]) * nrhs;
      poff[c] = ps;
      ps += i64(P) * nrhs;
    }
  p.xhat.reset(sizeof(double) * std::max<i64>(hs, 1));
  p.yhat.reset(sizeof(double) * std::max<i64>(hs, 1));
  p.xtil.reset(sizeof(double) * std::max<i64>(ps, 1));
  p.ytil.reset(sizeof(double) * std::max<i64>(ps, 1));
  const double* X = H.d_x.as<double>();
  double* xt = p.xt.as<double>();
  double* yt = p.yt.as<double>();
  double* xhat = p.xhat.as<double>();
  double* yhat = p.yhat.as<double>();
  double* xtil = H.identity_proj ? xhat : p.xtil.as<double>();
  double* ytil = H.identity_proj ? yhat : p.ytil.as<double>();
  const i64* til_off = H.identity_proj ? hoff.data() : poff.data();
  const double* basis = H.d_basis.as<double>();
  const double* transfer = H.d_transfer.as<double>();
  const double* proj = H.d_proj.as<double>();
  const double* nodes = H.d_nodes.as<double>();

  // Every block of right-hand sides is stored RHS-fastest (element (i, j) at
  // i nrhs + j), and every product is formed transposed, C^T = B^T A^T: the
  // right-hand sides are the rows of each output tile, so loads of them and
  // stores run along contiguous memory.
  const int N = int(nrhs);
  // close part: one item per leaf, one segment per near leaf, the leaf's
  // points along the output columns.  The kernel blocks are written out once
  // per plan and kept when they fit the budget (a stored operand runs at the
  // GEMM's rate); otherwise they are generated from the points inside the GEMM
  // for every product.
  std::vector<std::vector<int32_t>> nearOf(ncl);
  for (const Pair& pr : H.bt.near[0]) nearOf[pr.t].push_back(pr.s);
  const i64 f0 = tr.first_at_level(0), c0 = tr.count_at_level(0);
  std::vector<KernelBlock> kb;
  i64 kb_entries = 0;
  for (i64 t = f0; t < f0 + c0; ++t)
    for (int32_t s : nearOf[t]) {
      kb.push_back({kb_entries, int32_t(tr.start[t]), int32_t(tr.start[s]), int32_t(tr.size[t]), int32_t(tr.size[s]),
                    s == t ? 1 : 0, 0});
      kb_entries += tr.size[t] * tr.size[s];
    }
  const bool resident = close_blocks_fit(size_t(kb_entries) * sizeof(double));
  const double* blocks = nullptr;
  if (resident) {
    p.close_blocks.reset(sizeof(double) * std::max<i64>(kb_entries, 1));
    DeviceBuffer dkb = upload(kb);
    launch_kernel_blocks(dkb.as<KernelBlock>(), int(kb.size()), X, dim, H.kern, H.scale, H.diag, H.kparam,
                         p.close_blocks.as<double>(),
                         current_stream());
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(current_stream()));
    blocks = p.close_blocks.as<double>();
  }
  size_t b = 0;
  for (i64 t = f0; t < f0 + c0; ++t) {
    GemmItem& it = p.close.item(N, int(tr.size[t]), N, int(tr.size[t]));
    GemmBatch::set_out(it, 0, yt + tr.start[t] * nrhs, nrhs, false);
    for (int32_t s : nearOf[t]) {
      if (resident)
        p.close.seg(xt + tr.start[s] * nrhs, N, false, blocks + kb[b].off, int(tr.size[s]), false, int(tr.size[s]));
      else
        p.close.seg_genB(xt + tr.start[s] * nrhs, N, false, X + tr.start[t] * dim, X + tr.start[s] * dim, s == t,
                         int(tr.size[s]));
      ++b;
    }
  }
  // upward pass: xhat_t = R_t^T x_t at the leaves, sum of T_s^T xhat_s above
  p.up.resize(L + 1);
  for (int k = 0; k <= L; ++k) {
    const i64 f = tr.first_at_level(k), cnt = tr.count_at_level(k);
    for (i64 c = f; c < f + cnt; ++c) {
      if (!H.ff[c]) continue;
      const int r = H.rank[c];
      GemmItem& it = p.up[k].item(N, r, N, r);
      GemmBatch::set_out(it, 0, xhat + hoff[c], nrhs, false);
      if (k == 0) {
        p.up[k].seg(xt + tr.start[c] * nrhs, N, false, basis + H.basis_off[c], int(tr.size[c]), false,
                    int(tr.size[c]));
      } else {
        for (i64 s = 2 * c + 1; s <= 2 * c + 2; ++s)
          p.up[k].seg(xhat + hoff[s], N, false, transfer + H.transfer_off[s], H.rank[s], false, H.rank[s]);
      }
    }
  }
  // couplings: xtil = P^T xhat; ytil_t = sum_s K(nodes_t, nodes_s) xtil_s; yhat = P ytil
  std::vector<std::vector<int32_t>> farOf(ncl);
  for (const auto& lev : H.bt.far)
    for (const Pair& pr : lev) farOf[pr.t].push_back(pr.s);
  for (i64 c = 0; c < ncl; ++c) {
    if (!H.ff[c]) continue;
    const int r = H.rank[c];
    if (!H.identity_proj) {
      GemmItem& a = p.xproj.item(N, P, N, P);
      GemmBatch::set_out(a, 0, xtil + poff[c], nrhs, false);
      p.xproj.seg(xhat + hoff[c], N, false, proj + H.proj_off[c], r, false, r);
    }
    GemmItem& it = p.coup.item(N, P, N, P);
    GemmBatch::set_out(it, 0, ytil + til_off[c], nrhs, false);
    for (int32_t s : farOf[c])
      p.coup.seg_genB(xtil + til_off[s], N, false, nodes + c * i64(P) * dim, nodes + s * i64(P) * dim, false, P);
    if (!H.identity_proj) {
      GemmItem& b = p.yproj.item(N, r, N, r);
      GemmBatch::set_out(b, 0, yhat + hoff[c], nrhs, false);
      p.yproj.seg(ytil + poff[c], N, false, proj + H.proj_off[c], r, true, P);
    }
  }
  // downward pass: yhat_c += T_c yhat_father (levels L-1 .. 0)
  p.down.resize(L + 1);
  for (int k = L - 1; k >= 0; --k) {
    p.down[k].mode = GEMM_ADD;
    const i64 f = tr.first_at_level(k), cnt = tr.count_at_level(k);
    for (i64 c = f; c < f + cnt; ++c) {
      if (!H.ff[c] || !H.ff[(c - 1) / 2]) continue;
      const int r = H.rank[c], rp = H.rank[(c - 1) / 2];
      GemmItem& it = p.down[k].item(N, r, N, r);
      GemmBatch::set_out(it, 0, yhat + hoff[c], nrhs, false);
      p.down[k].seg(yhat + hoff[(c - 1) / 2], N, false, transfer + H.transfer_off[c], r, true, rp);
    }
  }
  p.leafout.mode = GEMM_ADD;
  for (i64 t = f0; t < f0 + c0; ++t) {
    if (!H.ff[t]) continue;
    const int r = H.rank[t];
    GemmItem& it = p.leafout.item(N, int(tr.size[t]), N, int(tr.size[t]));
    GemmBatch::set_out(it, 0, yt + tr.start[t] * nrhs, nrhs, false);
    p.leafout.seg(yhat + hoff[t], N, false, basis + H.basis_off[t], int(tr.size[t]), true, r);
  }
  std::vector<GemmBatch*> all{&p.close, &p.xproj, &p.coup, &p.yproj, &p.leafout};
  for (auto& g : p.up) all.push_back(&g);
  for (auto& g : p.down) all.push_back(&g);
  for (GemmBatch* g : all) {
    g->role = ROLE_MATVEC;
    g->prec = 0;
    g->set_generator(dim, H.kern, H.scale, H.diag, H.kparam);
  }
  upload_batches(all, p.desc);
  return mp;
}

// y_tree = A_H2 x_tree on plan buffers (x in p.xt, result in p.yt).
void run_matvec_tree(const h2_matrix& H, MatvecPlan& p, hipStream_t st) {
  p.graph.run(st, [&](hipStream_t s) {
    p.close.launch<double>(s);
    for (int k = 0; k <= H.tree.depth; ++k) p.up[k].launch<double>(s);
    p.xproj.launch<double>(s);
    p.coup.launch<double>(s);
    p.yproj.launch<double>(s);
    for (int k = H.tree.depth - 1; k >= 0; --k) p.down[k].launch<double>(s);
    p.leafout.launch<double>(s);
  });
}

MatvecPlan& matvec_plan(const h2_matrix& H, i64 nrhs);

}  // namespace h2

// The plan cache lives beside the handle (one plan per right-hand-side count).
// A matrix is used by one thread at a time; the map itself is shared.
static std::unordered_map<const h2_matrix*, std::unique_ptr<h2::MatvecPlan>> g_mv_plans;
static std::mutex g_mv_mu;

h2::MatvecPlan& h2::matvec_plan(const h2_matrix& H, i64 nrhs) {
  std::unique_ptr<h2::MatvecPlan>* slot;
  {
    std::lock_guard<std::mutex> lk(g_mv_mu);
    slot = &g_mv_plans[&H];  // node-based map: the slot stays valid
  }
  if (!*slot || (*slot)->nrhs != nrhs || (*slot)->tune_gen != tune_generation()) {
    slot->reset();
    *slot = make_matvec_plan(const_cast<h2_matrix&>(H), nrhs);
  }
  return **slot;
}

void h2_matrix_release_plans(const h2_matrix* H) {
  std::unique_ptr<h2::MatvecPlan> dead;
  {
    std::lock_guard<std::mutex> lk(g_mv_mu);
    auto it = g_mv_plans.find(H);
    if (it == g_mv_plans.end()) return;
    dead = std::move(it->second);
    g_mv_plans.erase(it);
  }
}

// ---------------------------------------------------------------- C ABI
namespace h2 {
std::string& last_error();
int status_of(const Error& e);
}  // namespace h2

#define H2_API_BEGIN try {
#define H2_API_END                                             \
  return H2_OK;                                                \
  }                                                            \
  catch (const h2::Error& e) {                                 \
    h2::last_error() = e.msg;                                  \
    return e.code;                                             \
  }                                                            \
  catch (const std::bad_alloc&) {                              \
    h2::last_error() = "host allocation failed";               \
    return H2_ENOMEM;                                          \
  }                                                            \
  catch (const std::exception& e) {                            \
    h2::last_error() = e.what();                               \
    return H2_EINVAL;                                          \
  }

extern "C" int h2_build(const double* pts, int64_t n, int dim, const h2_kernel* kernel,
                        const h2_build_opts* opts, h2_matrix** out) {
  H2_API_BEGIN
  if (!out) fail(H2_EINVAL, "null output handle");
  *out = nullptr;
  validate(pts, n, dim, kernel, opts);
  auto H = std::make_unique<h2_matrix>();
  fill_structure(*H, pts, n, dim, *kernel, *opts);
  check_duplicates(*H);
  if (opts->recompress_tol > 0 && opts->rank_cap < 0) fail(H2_EINVAL, "rank_cap must be >= 0");
  build_chebyshev(*H, opts->recompress_tol, opts->rank_cap);
  *out = H.release();
  H2_API_END
}

extern "C" int h2_import(const double* pts, int64_t n, int dim, const h2_kernel* kernel,
                         const h2_build_opts* opts, const int32_t* rank, const double* nodes,
                         const double* proj, const double* leaf_basis, const double* transfer,
                         h2_matrix** out) {
  H2_API_BEGIN
  if (!out) fail(H2_EINVAL, "null output handle");
  *out = nullptr;
  validate(pts, n, dim, kernel, opts);
  if (!rank || !nodes || !proj || !leaf_basis || !transfer) fail(H2_EINVAL, "null coefficient array");
  auto H = std::make_unique<h2_matrix>();
  fill_structure(*H, pts, n, dim, *kernel, *opts);
  check_duplicates(*H);
  const Tree& tr = H->tree;
  const i64 ncl = tr.ncl();
  const int P = H->P;
  H->rank.assign(rank, rank + ncl);
  for (i64 c = 0; c < ncl; ++c) {
    if ((H->rank[c] > 0) != bool(H->ff[c])) fail(H2_EINVAL, "rank > 0 must hold exactly for clusters with farfield");
    if (H->rank[c] > 64 || H->rank[c] < 0) fail(H2_EUNSUPPORTED, "rank must be in [0, 64]");
  }
  std::copy(nodes, nodes + size_t(ncl) * P * dim, H->nodes.begin());
  H->proj_off.assign(ncl, -1);
  H->basis_off.assign(ncl, -1);
  H->transfer_off.assign(ncl, -1);
  i64 po = 0, bo = 0, to = 0;
  for (i64 c = 0; c < ncl; ++c) {
    if (!H->ff[c]) continue;
    H->proj_off[c] = po;
    po += i64(H->rank[c]) * P;
    if (tr.is_leaf(c)) {
      H->basis_off[c] = bo;
      bo += tr.size[c] * H->rank[c];
    }
    if (c > 0 && H->ff[(c - 1) / 2]) {
      H->transfer_off[c] = to;
      to += i64(H->rank[c]) * H->rank[(c - 1) / 2];
    }
  }
  H->proj.assign(proj, proj + po);
  H->basis.assign(leaf_basis, leaf_basis + bo);
  H->transfer.assign(transfer, transfer + to);
  H->identity_proj = false;
  *out = H.release();
  H2_API_END
}

extern "C" int h2_matrix_info(const h2_matrix* h, int* depth, int64_t* ncl, int* cheb_points) {
  H2_API_BEGIN
  if (!h) fail(H2_EINVAL, "null handle");
  if (depth) *depth = h->tree.depth;
  if (ncl) *ncl = h->tree.ncl();
  if (cheb_points) *cheb_points = h->P;
  H2_API_END
}

extern "C" int h2_matrix_export_tree(const h2_matrix* h, int64_t* perm, int32_t* rank) {
  H2_API_BEGIN
  if (!h) fail(H2_EINVAL, "null handle");
  if (perm) std::copy(h->tree.perm.begin(), h->tree.perm.end(), perm);
  if (rank) std::copy(h->rank.begin(), h->rank.end(), rank);
  H2_API_END
}

extern "C" int h2_matvec(const h2_matrix* h, const double* x, double* y, int64_t nrhs, int64_t ld) {
  H2_API_BEGIN
  if (!h || !x || !y) fail(H2_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > 512 || ld < h->tree.n) fail(H2_EINVAL, "bad nrhs / ld");
  const i64 n = h->tree.n;
  MatvecPlan& p = matvec_plan(*h, nrhs);
  hipStream_t st = current_stream();
  launch_gather_rm(x, ld, h->d_perm.as<i64>(), p.xt.as<double>(), n, nrhs, st);
  run_matvec_tree(*h, p, st);
  launch_scatter_rm(p.yt.as<double>(), h->d_perm.as<i64>(), y, ld, n, nrhs, st);
  HIPCHECK(hipGetLastError());
  H2_API_END
}

extern "C" void h2_matrix_destroy(h2_matrix* h) {
  if (!h) return;
  (void)hipStreamSynchronize(current_stream());
  h2_matrix_release_plans(h);
  delete h;
}

namespace h2 {
struct MatvecPlanView {
  double* xt;
  double* yt;
};
MatvecPlanView matvec_buffers(MatvecPlan& p) { return {p.xt.as<double>(), p.yt.as<double>()}; }
}  // namespace h2
