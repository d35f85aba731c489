// C ABI of libh2sp: sparsification, factorisation and solve entry points.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>

#include <omp.h>

#include "factor.h"

namespace h2 {
h2_factor* factor(h2_sparse* sp, int mode, double tau, hipStream_t st, double* phase_ms, bool level_events);
void analyze_fill(const h2_sparse& sp, double* entries, double* flops);
void set_stream(hipStream_t s);
std::string& last_error() {
  static thread_local std::string msg;
  return msg;
}
static thread_local double g_timings[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
static thread_local double g_work[20] = {0};
}  // namespace h2

int apply_inverse_impl(h2_factor* f, const double* b, double* x, h2::i64 nrhs, h2::i64 ld);
int solve_impl(h2_factor* f, const double* b, double* x, h2::i64 nrhs, h2::i64 ld, const h2_solve_opts* o,
               h2_solve_info* info);
int solve_with_impl(const h2_matrix* A, h2_factor* f, const double* b, double* x, h2::i64 nrhs, h2::i64 ld,
                    const h2_solve_opts* o, h2_solve_info* info);

using namespace h2;

#define H2_API_BEGIN try {
#define H2_API_END                               \
  return H2_OK;                                  \
  }                                              \
  catch (const h2::Error& e) {                   \
    h2::last_error() = e.msg;                    \
    return e.code;                               \
  }                                              \
  catch (const std::bad_alloc&) {                \
    h2::last_error() = "host allocation failed"; \
    return H2_ENOMEM;                            \
  }                                              \
  catch (const std::exception& e) {              \
    h2::last_error() = e.what();                 \
    return H2_EINVAL;                            \
  }



extern "C" const char* h2_last_error(void) { return h2::last_error().c_str(); }

extern "C" int h2_set_stream(void* stream) {
  h2::set_stream(static_cast<hipStream_t>(stream));
  return H2_OK;
}

// After the sweep: only Q_t (for U and V) and S outlive it; the plan's work
// counts go to h2_last_work (summed over a batch).
static void finish_sparsify(h2_sparse& sp) {
  for (int side = 0; side < 2; ++side) {
    sp.dC[side].reset(0);
    sp.dG[side].reset(0);
  }
  sp.dTmp.reset(0);
  sp.dB.reset(0);
  sp.dW.reset(0);
  sp.dWt.reset(0);
  sp.dRhat.reset(0);
  sp.dDesc.reset(0);
  sp.levels.clear();
  const PlanCounts& pc = sp.counts;
  g_work[0] += pc.flops_qr + pc.flops_misc;
  g_work[1] += pc.flops_close;
  g_work[2] += pc.flops_coup;
  g_work[3] += pc.flops_strip;
  g_work[6] += pc.bytes_qr;
}

// Runs job(i) for i < count on a pool of host threads, each with a stream of
// its own (so that the instances' device work overlaps), then makes the
// caller's stream wait for all of them.  The first error is rethrown.
static void run_pooled(int count, const std::function<void(int)>& job) {
  const hipStream_t caller = current_stream();
  const int nthr = std::max(1, std::min(count, 8));
  const int omp_share = std::max(1, omp_get_max_threads() / nthr);
  std::vector<hipStream_t> streams(nthr, nullptr);
  hipEvent_t ready;
  HIPCHECK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  HIPCHECK(hipEventRecord(ready, caller));
  for (auto& st : streams) {
    HIPCHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    HIPCHECK(hipStreamWaitEvent(st, ready, 0));  // inputs written on the caller's stream
  }
  std::atomic<int> next{0};
  std::mutex mu;
  int code = 0;
  std::string msg;
  std::vector<std::thread> pool;
  for (int t = 0; t < nthr; ++t)
    pool.emplace_back([&, t] {
      set_stream(streams[t]);
      omp_set_num_threads(omp_share);
      for (int i = next++; i < count; i = next++) {
        try {
          job(i);
        } catch (const Error& e) {
          std::lock_guard<std::mutex> lk(mu);
          if (!code) code = e.code, msg = e.msg;
        } catch (const std::bad_alloc&) {
          std::lock_guard<std::mutex> lk(mu);
          if (!code) code = H2_ENOMEM, msg = "host allocation failed";
        } catch (const std::exception& e) {
          std::lock_guard<std::mutex> lk(mu);
          if (!code) code = H2_EINVAL, msg = e.what();
        }
      }
      (void)hipStreamSynchronize(streams[t]);
    });
  for (auto& th : pool) th.join();
  for (auto& st : streams) (void)hipStreamDestroy(st);
  (void)hipEventDestroy(ready);
  if (code) fail(code, msg);
}

extern "C" int h2_sparsify(h2_matrix* h, const h2_sparsify_opts* opts, h2_sparse** out) {
  H2_API_BEGIN
  if (!h || !out) fail(H2_EINVAL, "null argument");
  *out = nullptr;
  const int prec = opts ? opts->precision : H2_FP64;
  if (prec != H2_FP64 && prec != H2_MIXED) fail(H2_EINVAL, "unknown precision");
  std::unique_ptr<h2_sparse> sp(plan_sparsify(h, prec, true));
  std::fill(g_timings, g_timings + 12, 0.0);
  std::fill(g_work, g_work + 20, 0.0);
  run_sparsify(*sp, current_stream(), g_timings);
  HIPCHECK(hipStreamSynchronize(current_stream()));
  finish_sparsify(*sp);
  HIPCHECK(hipStreamSynchronize(current_stream()));
  *out = sp.release();
  H2_API_END
}

extern "C" int h2_sparse_info(const h2_sparse* sp, int64_t* nnz_blocks, int64_t* nnz_entries) {
  H2_API_BEGIN
  if (!sp) fail(H2_EINVAL, "null handle");
  if (nnz_blocks) *nnz_blocks = int64_t(sp->colidx.size());
  if (nnz_entries) *nnz_entries = sp->s_entries;
  H2_API_END
}

extern "C" int h2_sparse_export_plan(const h2_sparse* sp, int64_t* n_act, int64_t* kept, int64_t* nonbasis,
                                     int64_t* soff, int64_t* elim, int64_t* rowptr, int64_t* colidx) {
  H2_API_BEGIN
  if (!sp) fail(H2_EINVAL, "null handle");
  auto cp = [](const std::vector<i64>& v, int64_t* dst) {
    if (dst) std::copy(v.begin(), v.end(), dst);
  };
  cp(sp->n_act, n_act);
  cp(sp->kept, kept);
  cp(sp->nonbasis, nonbasis);
  cp(sp->soff, soff);
  cp(sp->eorder, elim);
  cp(sp->rowptr, rowptr);
  cp(sp->colidx, colidx);
  H2_API_END
}

extern "C" int h2_sparse_export_block(const h2_sparse* sp, int64_t t, int64_t s, double* out) {
  H2_API_BEGIN
  if (!sp || !out) fail(H2_EINVAL, "null argument");
  if (t < 0 || s < 0 || t >= sp->ncl || s >= sp->ncl) fail(H2_EINVAL, "cluster out of range");
  i64 b = sp->block_of(t, s);
  const bool transposed = b < 0;
  if (transposed) b = sp->block_of(s, t);
  if (b < 0) fail(H2_EINVAL, "no such block in the pattern of S");
  const i64 mt = sp->nonbasis[t], ms = sp->nonbasis[s], cnt = mt * ms;
  HIPCHECK(hipStreamSynchronize(current_stream()));
  std::vector<double> tmp(cnt);
  if (sp->precision == H2_MIXED) {
    std::vector<float> tf(cnt);
    HIPCHECK(hipMemcpy(tf.data(), sp->dS.as<float>() + sp->blk_off[b], sizeof(float) * cnt, hipMemcpyDeviceToHost));
    for (i64 i = 0; i < cnt; ++i) tmp[i] = tf[i];
  } else {
    HIPCHECK(hipMemcpy(tmp.data(), sp->dS.as<double>() + sp->blk_off[b], sizeof(double) * cnt, hipMemcpyDeviceToHost));
  }
  // stored block is m_t x m_s (or m_s x m_t when transposed), column-major
  for (i64 j = 0; j < ms; ++j)
    for (i64 i = 0; i < mt; ++i) out[i + j * mt] = transposed ? tmp[j + i * ms] : tmp[i + j * mt];
  H2_API_END
}

extern "C" int h2_sparse_export_q(const h2_sparse* sp, int64_t t, double* out) {
  H2_API_BEGIN
  if (!sp || !out) fail(H2_EINVAL, "null argument");
  if (t < 0 || t >= sp->ncl || sp->q_off[t] < 0) fail(H2_EINVAL, "cluster has no Q");
  HIPCHECK(hipStreamSynchronize(current_stream()));
  HIPCHECK(hipMemcpy(out, sp->dQ.as<double>() + sp->q_off[t], sizeof(double) * sp->n_act[t] * sp->n_act[t],
                     hipMemcpyDeviceToHost));
  H2_API_END
}

extern "C" int h2_factor_S(h2_sparse* sp, const h2_factor_opts* opts, h2_factor** out) {
  H2_API_BEGIN
  if (!sp || !out) fail(H2_EINVAL, "null argument");
  *out = nullptr;
  const int mode = opts ? opts->mode : H2_FACTOR_ILU0;
  const double tau = opts ? opts->tau : 0.0;
  if (mode != H2_FACTOR_EXACT && mode != H2_FACTOR_ILU0 && mode != H2_FACTOR_ILUT)
    fail(H2_EINVAL, "unknown factorisation mode");
  if (mode == H2_FACTOR_ILUT && !(tau >= 0.0)) fail(H2_EINVAL, "ILUt drop tolerance must be >= 0");
  if (sp->factored) fail(H2_EINVAL, "S of this sparse handle is already factored");
  for (int i = 4; i < 12; ++i) g_timings[i] = 0;
  double ph[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  std::unique_ptr<h2_factor> f(factor(sp, mode, tau, current_stream(), ph, true));
  g_timings[4] = ph[4];
  g_timings[5] = ph[5];
  g_timings[7] = ph[6];
  for (int c = 0; c < 3; ++c) g_timings[8 + c] = ph[7 + c];
  g_work[4] = f->flops_inv + f->flops_z;
  g_work[5] = f->flops_schur;
  g_work[7] = double(f->split_targets);
  g_work[8] = double(f->schur_launches);
  g_work[9] = double(sp->s_entries);
  for (int c = 0; c < 3; ++c) {
    g_work[10 + 2 * c] = f->flops_cls[c];
    g_work[11 + 2 * c] = double(f->launches_cls[c]);
  }
  g_work[16] = double(f->ilut_dropped);
  g_work[17] = double(f->ilut_kept);
  *out = f.release();
  H2_API_END
}

extern "C" int h2_plan_report(h2_matrix* h, int with_fill, h2_plan_counts* out) {
  H2_API_BEGIN
  if (!h || !out) fail(H2_EINVAL, "null argument");
  std::unique_ptr<h2_sparse> sp(plan_symbolic(h));
  const Tree& tr = h->tree;
  h2_plan_counts r{};
  r.n = tr.n;
  r.clusters = tr.ncl();
  r.depth = tr.depth;
  r.s_blocks = i64(sp->colidx.size());
  r.s_upper_entries = sp->s_entries;
  i64 diag = 0;
  for (i64 c = 0; c < sp->ncl; ++c) diag += sp->nonbasis[c] * sp->nonbasis[c];
  r.s_entries = 2 * sp->s_entries - diag;
  r.q_entries = sp->q_entries;
  i64 h2e = 0, close = 0;
  for (i64 c = 0; c < tr.ncl(); ++c) {
    if (h->basis_off.size() > size_t(c) && h->basis_off[c] >= 0) h2e += tr.size[c] * i64(h->rank[c]);
    if (h->transfer_off.size() > size_t(c) && h->transfer_off[c] >= 0 && c > 0)
      h2e += i64(h->rank[c]) * h->rank[(c - 1) / 2];
  }
  for (const auto& lv : h->bt.far)
    for (const Pair& p : lv) h2e += i64(h->rank[p.t]) * h->rank[p.s];
  if (!h->bt.near.empty())
    for (const Pair& p : h->bt.near[0]) close += tr.size[p.t] * tr.size[p.s];
  r.h2_entries = h2e + close;
  r.h2_close_entries = close;
  r.filled_entries = -1;
  r.exact_flops = -1;
  if (with_fill) {
    double e = 0, fl = 0;
    analyze_fill(*sp, &e, &fl);
    r.filled_entries = int64_t(e);
    r.exact_flops = fl;
  }
  *out = r;
  H2_API_END
}

extern "C" int h2_factor_analyze(const h2_sparse* sp, int64_t* filled_entries, double* exact_flops) {
  H2_API_BEGIN
  if (!sp) fail(H2_EINVAL, "null argument");
  if (sp->factored) fail(H2_EINVAL, "S of this sparse handle is already factored");
  double e = 0, fl = 0;
  analyze_fill(*sp, &e, &fl);
  if (filled_entries) *filled_entries = int64_t(e);
  if (exact_flops) *exact_flops = fl;
  H2_API_END
}

extern "C" int h2_sparsify_batch(h2_matrix* const* hs, int count, const h2_sparsify_opts* opts, h2_sparse** outs) {
  H2_API_BEGIN
  if (!hs || !outs || count < 1) fail(H2_EINVAL, "null argument or empty batch");
  for (int i = 0; i < count; ++i) {
    if (!hs[i]) fail(H2_EINVAL, "null matrix in the batch");
    // instances are planned on concurrent threads, and planning uploads the
    // matrix's device copy: one matrix may appear once
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) fail(H2_EINVAL, "the same matrix twice in the batch");
    outs[i] = nullptr;
  }
  // the merged sweep generates every instance's close blocks in one launch
  for (int i = 1; i < count; ++i)
    if (hs[i]->kern != hs[0]->kern || hs[i]->kparam != hs[0]->kparam)
      fail(H2_EUNSUPPORTED, "batched sparsification of matrices of different kernels");
  const int prec = opts ? opts->precision : H2_FP64;
  if (prec != H2_FP64 && prec != H2_MIXED) fail(H2_EINVAL, "unknown precision");
  std::vector<std::unique_ptr<h2_sparse>> own(count);
  std::vector<h2_sparse*> sps(count);
  // the instances are planned concurrently (host work); their sweeps are merged below
  run_pooled(count, [&](int i) { own[i].reset(plan_sparsify(hs[i], prec, false)); });
  for (int i = 0; i < count; ++i) sps[i] = own[i].get();
  std::fill(g_timings, g_timings + 12, 0.0);
  std::fill(g_work, g_work + 20, 0.0);
  run_sparsify_batch(sps, current_stream(), g_timings);
  HIPCHECK(hipStreamSynchronize(current_stream()));
  for (int i = 0; i < count; ++i) {
    finish_sparsify(*own[i]);
    outs[i] = own[i].release();
  }
  H2_API_END
}

extern "C" int h2_factor_S_batch(h2_sparse* const* sps, int count, const h2_factor_opts* opts, h2_factor** outs) {
  H2_API_BEGIN
  if (!sps || !outs || count < 1) fail(H2_EINVAL, "null argument or empty batch");
  const int mode = opts ? opts->mode : H2_FACTOR_ILU0;
  const double tau = opts ? opts->tau : 0.0;
  if (mode != H2_FACTOR_EXACT && mode != H2_FACTOR_ILU0 && mode != H2_FACTOR_ILUT)
    fail(H2_EINVAL, "unknown factorisation mode");
  if (mode == H2_FACTOR_ILUT && !(tau >= 0.0)) fail(H2_EINVAL, "ILUt drop tolerance must be >= 0");
  for (int i = 0; i < count; ++i) {
    if (!sps[i]) fail(H2_EINVAL, "null sparse handle in the batch");
    if (sps[i]->factored) fail(H2_EINVAL, "S of a sparse handle in the batch is already factored");
    for (int j = 0; j < i; ++j)
      if (sps[j] == sps[i]) fail(H2_EINVAL, "the same sparse handle twice in the batch");
    outs[i] = nullptr;
  }
  std::vector<std::unique_ptr<h2_factor>> fs(count);
  std::vector<double> ph(size_t(count) * 10, 0.0);
  run_pooled(count, [&](int i) {
    fs[i].reset(factor(sps[i], mode, tau, current_stream(), &ph[size_t(i) * 10], false));
  });
  std::fill(g_timings + 4, g_timings + 12, 0.0);
  std::fill(g_work + 4, g_work + 20, 0.0);
  for (int i = 0; i < count; ++i) {
    g_timings[4] += ph[size_t(i) * 10 + 4];
    g_timings[5] += ph[size_t(i) * 10 + 5];
    for (int c = 0; c < 3; ++c) g_timings[8 + c] += ph[size_t(i) * 10 + 7 + c];
    g_work[4] += fs[i]->flops_inv + fs[i]->flops_z;
    g_work[5] += fs[i]->flops_schur;
    g_work[7] += double(fs[i]->split_targets);
    g_work[8] += double(fs[i]->schur_launches);
    g_work[9] += double(sps[i]->s_entries);
    for (int c = 0; c < 3; ++c) {
      g_work[10 + 2 * c] += fs[i]->flops_cls[c];
      g_work[11 + 2 * c] += double(fs[i]->launches_cls[c]);
    }
    g_work[16] += double(fs[i]->ilut_dropped);
    g_work[17] += double(fs[i]->ilut_kept);
  }
  for (int i = 0; i < count; ++i) outs[i] = fs[i].release();
  H2_API_END
}

extern "C" int h2_solve_batch(h2_factor* const* fs, int count, const double* const* b, double* const* x,
                              const int64_t* nrhs, const int64_t* ld, const h2_solve_opts* opts,
                              h2_solve_info* infos) {
  H2_API_BEGIN
  if (!fs || !b || !x || !nrhs || !ld || count < 1) fail(H2_EINVAL, "null argument or empty batch");
  for (int i = 0; i < count; ++i) {
    if (!fs[i] || !b[i] || !x[i]) fail(H2_EINVAL, "null factor or vector in the batch");
    if (nrhs[i] < 1 || nrhs[i] > 512 || ld[i] < fs[i]->sp->H->tree.n) fail(H2_EINVAL, "bad nrhs / ld in the batch");
    // the instances run on concurrent threads, and a matrix keeps one
    // matvec plan (its vectors included): one matrix may appear once
    for (int j = 0; j < i; ++j) {
      if (fs[j] == fs[i]) fail(H2_EINVAL, "the same factor twice in the batch");
      if (fs[j]->sp->H == fs[i]->sp->H) fail(H2_EINVAL, "two factors of the same matrix in the batch");
    }
  }
  std::vector<int> rc(count, H2_OK);
  run_pooled(count, [&](int i) {
    rc[i] = solve_impl(fs[i], b[i], x[i], nrhs[i], ld[i], opts, infos ? &infos[i] : nullptr);
  });
  for (int i = 0; i < count; ++i)
    if (rc[i] == H2_ENOCONV) fail(H2_ENOCONV, "refinement stopped above the tolerance (instance " + std::to_string(i) + ")");
  H2_API_END
}

extern "C" int h2_solve(h2_factor* f, const double* b, double* x, int64_t nrhs, int64_t ld,
                        const h2_solve_opts* opts, h2_solve_info* info) {
  H2_API_BEGIN
  if (!f || !b || !x) fail(H2_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > 512 || ld < f->sp->H->tree.n) fail(H2_EINVAL, "bad nrhs / ld");
  const int rc = solve_impl(f, b, x, nrhs, ld, opts, info);
  if (rc == H2_ENOCONV) fail(H2_ENOCONV, "solve stopped above the tolerance");
  H2_API_END
}

extern "C" int h2_solve_with(const h2_matrix* a, h2_factor* f, const double* b, double* x, int64_t nrhs,
                             int64_t ld, const h2_solve_opts* opts, h2_solve_info* info) {
  H2_API_BEGIN
  if (!a || !f || !b || !x) fail(H2_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > 512 || ld < a->tree.n) fail(H2_EINVAL, "bad nrhs / ld");
  const int rc = solve_with_impl(a, f, b, x, nrhs, ld, opts, info);
  if (rc == H2_ENOCONV) fail(H2_ENOCONV, "solve stopped above the tolerance");
  H2_API_END
}

extern "C" int h2_apply_inverse(h2_factor* f, const double* b, double* x, int64_t nrhs, int64_t ld) {
  H2_API_BEGIN
  if (!f || !b || !x) fail(H2_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > 512 || ld < f->sp->H->tree.n) fail(H2_EINVAL, "bad nrhs / ld");
  apply_inverse_impl(f, b, x, nrhs, ld);
  H2_API_END
}

int apply_inverse_noalloc_impl(h2_factor* f, const double* b, double* x, h2::i64 nrhs, h2::i64 ld);

extern "C" int h2_apply_inverse_noalloc(h2_factor* f, const double* b, double* x, int64_t nrhs, int64_t ld) {
  H2_API_BEGIN
  if (!f || !b || !x) fail(H2_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > 512 || ld < f->sp->H->tree.n) fail(H2_EINVAL, "bad nrhs / ld");
  apply_inverse_noalloc_impl(f, b, x, nrhs, ld);
  H2_API_END
}

extern "C" int h2_last_timings(double* ms, int count) {
  H2_API_BEGIN
  if (!ms) fail(H2_EINVAL, "null argument");
  // [6] reports the sparsify total, [7] (internal) the factor total
  for (int i = 0; i < count && i < 12; ++i) ms[i] = g_timings[i];
  H2_API_END
}

extern "C" int h2_last_work(double* work, int count) {
  H2_API_BEGIN
  if (!work) fail(H2_EINVAL, "null argument");
  for (int i = 0; i < count && i < 20; ++i) work[i] = g_work[i];
  H2_API_END
}

extern "C" void h2_sparse_destroy(h2_sparse* sp) {
  if (!sp) return;
  (void)hipStreamSynchronize(current_stream());
  delete sp;
}

extern "C" void h2_factor_destroy(h2_factor* f) {
  if (!f) return;
  (void)hipStreamSynchronize(current_stream());
  delete f;
}
