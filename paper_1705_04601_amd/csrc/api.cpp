// C ABI of libh2sp: sparsification, factorisation and solve entry points.
#include <cstring>
#include <memory>

#include "factor.h"

namespace h2 {
h2_sparse* plan_sparsify(h2_matrix* H, int precision);
h2_factor* factor(h2_sparse* sp, bool exact, hipStream_t st, double* phase_ms);
void analyze_fill(const h2_sparse& sp, double* entries, double* flops);
void set_stream(hipStream_t s);
std::string& last_error() {
  static thread_local std::string msg;
  return msg;
}
static thread_local double g_timings[8] = {0, 0, 0, 0, 0, 0, 0, 0};
static thread_local double g_work[16] = {0};
}  // namespace h2

int apply_inverse_impl(h2_factor* f, const double* b, double* x, h2::i64 nrhs, h2::i64 ld);
int solve_impl(h2_factor* f, const double* b, double* x, h2::i64 nrhs, h2::i64 ld, const h2_solve_opts* o,
               h2_solve_info* info);

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

extern "C" int h2_sparsify(h2_matrix* h, const h2_sparsify_opts* opts, h2_sparse** out) {
  H2_API_BEGIN
  if (!h || !out) fail(H2_EINVAL, "null argument");
  *out = nullptr;
  const int prec = opts ? opts->precision : H2_FP64;
  if (prec != H2_FP64 && prec != H2_MIXED) fail(H2_EINVAL, "unknown precision");
  std::unique_ptr<h2_sparse> sp(plan_sparsify(h, prec));
  std::fill(g_timings, g_timings + 8, 0.0);
  run_sparsify(*sp, current_stream(), g_timings);
  HIPCHECK(hipStreamSynchronize(current_stream()));
  // only Q_t (for U and V) and S outlive the sweep
  for (int side = 0; side < 2; ++side) {
    sp->dC[side].reset(0);
    sp->dG[side].reset(0);
  }
  sp->dTmp.reset(0);
  sp->dB.reset(0);
  sp->dW.reset(0);
  sp->dWt.reset(0);
  sp->dRhat.reset(0);
  sp->dDesc.reset(0);
  sp->levels.clear();
  const PlanCounts& pc = sp->counts;
  g_work[0] = pc.flops_qr + pc.flops_misc;
  g_work[1] = pc.flops_close;
  g_work[2] = pc.flops_coup;
  g_work[3] = pc.flops_strip;
  g_work[6] = pc.bytes_qr;
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
  if (mode != H2_FACTOR_EXACT && mode != H2_FACTOR_ILU0) fail(H2_EINVAL, "unknown factorisation mode");
  if (sp->factored) fail(H2_EINVAL, "S of this sparse handle is already factored");
  for (int i = 4; i < 8; ++i) g_timings[i] = 0;
  double ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::unique_ptr<h2_factor> f(factor(sp, mode == H2_FACTOR_EXACT, current_stream(), ph));
  g_timings[4] = ph[4];
  g_timings[5] = ph[5];
  g_timings[7] = ph[6];
  g_work[4] = f->flops_inv + f->flops_z;
  g_work[5] = f->flops_schur;
  g_work[7] = double(f->split_targets);
  g_work[8] = double(f->schur_launches);
  g_work[9] = double(sp->s_entries);
  *out = f.release();
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

extern "C" int h2_solve(h2_factor* f, const double* b, double* x, int64_t nrhs, int64_t ld,
                        const h2_solve_opts* opts, h2_solve_info* info) {
  H2_API_BEGIN
  if (!f || !b || !x) fail(H2_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > 512 || ld < f->sp->H->tree.n) fail(H2_EINVAL, "bad nrhs / ld");
  const int rc = solve_impl(f, b, x, nrhs, ld, opts, info);
  if (rc == H2_ENOCONV) fail(H2_ENOCONV, "refinement stopped above the tolerance");
  H2_API_END
}

extern "C" int h2_apply_inverse(h2_factor* f, const double* b, double* x, int64_t nrhs, int64_t ld) {
  H2_API_BEGIN
  if (!f || !b || !x) fail(H2_EINVAL, "null argument");
  if (nrhs < 1 || nrhs > 512 || ld < f->sp->H->tree.n) fail(H2_EINVAL, "bad nrhs / ld");
  apply_inverse_impl(f, b, x, nrhs, ld);
  H2_API_END
}

extern "C" int h2_last_timings(double* ms, int count) {
  H2_API_BEGIN
  if (!ms) fail(H2_EINVAL, "null argument");
  // [6] reports the sparsify total, [7] (internal) the factor total
  double tmp[8];
  std::copy(g_timings, g_timings + 8, tmp);
  for (int i = 0; i < count && i < 8; ++i) ms[i] = tmp[i];
  H2_API_END
}

extern "C" int h2_last_work(double* work, int count) {
  H2_API_BEGIN
  if (!work) fail(H2_EINVAL, "null argument");
  for (int i = 0; i < count && i < 16; ++i) work[i] = g_work[i];
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
