// Autotuner: measures the built tile shapes of every GEMM kind a workload
// plans, and the knobs of the Schur work lists, on the caller's own matrix,
// and keeps the fastest of each in the tuning table (then in the JSON cache).
// A client of the library's own entry points: each trial runs the real
// sparsification, factorisation, preconditioner application or product and
// reads its device time (HIP events inside the library) or, for the
// application and the product, the time of the synchronous call.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "h2_internal.h"
#include "h2sp.h"
#include "kernels.h"
#include "tune.h"

namespace h2 {
std::string& last_error();  // message of the last failed call on this thread (api.cpp)
namespace {

void check(int code) {
  if (code != H2_OK) fail(code, h2_last_error());
}

double wall_ms(const std::function<void()>& fn) {
  const auto t0 = std::chrono::steady_clock::now();
  fn();
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// GEMM entries of one role ("transform", "factor", "solve", "matvec") that
// the runs since the last tune_reset_used used.
std::vector<std::string> used_keys(const std::string& role) {
  std::vector<std::string> out;
  const std::string rep = tune_report();
  const size_t u = rep.find("\"used\": {");
  size_t i = u == std::string::npos ? rep.size() : u + 9;
  while (i < rep.size()) {
    const size_t a = rep.find('"', i);
    if (a == std::string::npos) break;
    const size_t b = rep.find('"', a + 1);
    const std::string k = rep.substr(a + 1, b - a - 1);
    if (k.compare(0, 5, "gemm.") == 0 && k.find("." + role + ".") != std::string::npos) out.push_back(k);
    i = rep.find(',', b);
    if (i == std::string::npos) break;
  }
  return out;
}

// The built variants of a GEMM key.
std::vector<int64_t> variants_of(const std::string& key) {
  char p[8] = {0}, r[16] = {0};
  int am = 0, bm = 0, m = 0;
  std::vector<int64_t> out;
  if (std::sscanf(key.c_str(), "gemm.%3[f0-9].%15[a-z].a%db%d.m%d", p, r, &am, &bm, &m) != 5) return out;
  const int prec = std::string(p) == "f32" ? 1 : 0;
  const std::string rs(r);
  const int role = rs == "factor" ? ROLE_FACTOR : rs == "solve" ? ROLE_SOLVE : rs == "matvec" ? ROLE_MATVEC
                                                                                               : ROLE_TRANSFORM;
  for (int v = 0; v < kGemmVariants; ++v)
    if (gemm_shape(prec, role, am, bm, v) != 0) out.push_back(v);
  return out;
}

// Coordinate step: every candidate of one key with the others fixed; the
// fastest (minimum over `reps` runs) stays in the table.
void descend(const std::string& key, const std::vector<int64_t>& cands, int reps,
             const std::function<double()>& measure, std::string& log) {
  if (cands.size() < 2) return;
  int64_t best = cands[0];
  double best_ms = 1e300;
  char line[256];
  for (int64_t v : cands) {
    tune_set(key, v);
    double ms = 1e300;
    for (int r = 0; r < reps; ++r) ms = std::min(ms, measure());
    std::snprintf(line, sizeof line, "%s = %lld: %.3f ms\n", key.c_str(), (long long)v, ms);
    log += line;
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  tune_set(key, best);
  std::snprintf(line, sizeof line, "%s -> %lld\n", key.c_str(), (long long)best);
  log += line;
}

}  // namespace
}  // namespace h2

using namespace h2;

extern "C" int h2_autotune(h2_matrix* h, int precision, int64_t nrhs, const char* path) {
  try {
    if (!h || nrhs < 1 || nrhs > 512) fail(H2_EINVAL, "autotune: null matrix or nrhs outside 1..512");
    if (precision != H2_FP64 && precision != H2_MIXED) fail(H2_EINVAL, "autotune: unknown precision");
    const bool trace = trace_level() > 0;
    std::string log;
    const i64 n = h->tree.n;
    hipStream_t st = current_stream();
    DeviceBuffer b(sizeof(double) * n * nrhs), x(sizeof(double) * n * nrhs);
    launch_fill(b.as<double>(), n * nrhs, 1.0, st);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));
    h2_sparsify_opts so{precision};
    h2_factor_opts fo{};
    fo.mode = H2_FACTOR_ILU0;
    double ms[12];
    auto sparsify_ms = [&]() {
      h2_sparse* sp = nullptr;
      check(h2_sparsify(h, &so, &sp));
      check(h2_last_timings(ms, 12));
      h2_sparse_destroy(sp);
      return ms[6];
    };
    auto factor_ms = [&]() {
      h2_sparse* sp = nullptr;
      h2_factor* f = nullptr;
      check(h2_sparsify(h, &so, &sp));
      const int code = h2_factor_S(sp, &fo, &f);
      if (code != H2_OK) {
        h2_sparse_destroy(sp);
        check(code);
      }
      check(h2_last_timings(ms, 12));
      h2_factor_destroy(f);
      h2_sparse_destroy(sp);
      return ms[7];
    };
    // the sparsification's GEMMs
    tune_reset_used();
    sparsify_ms();
    for (const std::string& k : used_keys("transform")) descend(k, variants_of(k), 2, sparsify_ms, log);
    // the factorisation's GEMMs and the Schur work lists
    tune_reset_used();
    factor_ms();
    for (const std::string& k : used_keys("factor")) descend(k, variants_of(k), 1, factor_ms, log);
    descend("schur.split_k", {256, 512, 1024, 2048}, 1, factor_ms, log);
    descend("schur.key_z", {0, 1}, 1, factor_ms, log);
    descend("schur.split_big", {0, 1}, 1, factor_ms, log);
    // the preconditioner application's sweeps (one warm-up call plans them)
    {
      h2_sparse* sp = nullptr;
      h2_factor* f = nullptr;
      check(h2_sparsify(h, &so, &sp));
      const int code = h2_factor_S(sp, &fo, &f);
      if (code != H2_OK) {
        h2_sparse_destroy(sp);
        check(code);
      }
      auto apply_ms = [&]() {
        check(h2_apply_inverse(f, b.as<double>(), x.as<double>(), nrhs, n));
        return wall_ms([&] { check(h2_apply_inverse(f, b.as<double>(), x.as<double>(), nrhs, n)); });
      };
      try {
        tune_reset_used();
        apply_ms();
        for (const std::string& k : used_keys("solve")) descend(k, variants_of(k), 3, apply_ms, log);
        descend("solve.split_k", {512, 1024, 2048, 4096, int64_t(1) << 30}, 3, apply_ms, log);
      } catch (...) {
        h2_factor_destroy(f);
        h2_sparse_destroy(sp);
        throw;
      }
      h2_factor_destroy(f);
      h2_sparse_destroy(sp);
    }
    // the FP64 product
    {
      DeviceBuffer y(sizeof(double) * n * nrhs);
      auto matvec_ms = [&]() {
        check(h2_matvec(h, b.as<double>(), y.as<double>(), nrhs, n));
        HIPCHECK(hipStreamSynchronize(st));
        return wall_ms([&] {
          check(h2_matvec(h, b.as<double>(), y.as<double>(), nrhs, n));
          HIPCHECK(hipStreamSynchronize(st));
        });
      };
      tune_reset_used();
      matvec_ms();
      for (const std::string& k : used_keys("matvec")) descend(k, variants_of(k), 3, matvec_ms, log);
    }
    if (trace) std::fprintf(stderr, "[h2sp] autotune (%s, %lld rhs):\n%s", precision == H2_MIXED ? "mixed" : "fp64",
                            (long long)nrhs, log.c_str());
    if (path) tune_save(path);
    return H2_OK;
  } catch (const Error& e) {
    last_error() = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    last_error() = "host allocation failed";
    return H2_ENOMEM;
  } catch (const std::exception& e) {
    last_error() = e.what();
    return H2_EINVAL;
  }
}

extern "C" int h2_tune_set(const char* key, int64_t value) {
  try {
    if (!key) fail(H2_EINVAL, "null key");
    tune_set(key, value);
    return H2_OK;
  } catch (const Error& e) {
    last_error() = e.msg;
    return e.code;
  }
}

extern "C" int h2_tune_get(const char* key, int64_t* value) {
  try {
    if (!key || !value) fail(H2_EINVAL, "null argument");
    if (!tune_get(key, value)) fail(H2_EINVAL, std::string("no tuning entry ") + key);
    return H2_OK;
  } catch (const Error& e) {
    last_error() = e.msg;
    return e.code;
  }
}

extern "C" int h2_tune_clear(void) {
  tune_clear();
  return H2_OK;
}

extern "C" int h2_tune_load(const char* path) {
  try {
    tune_load(path ? path : "");
    return H2_OK;
  } catch (const Error& e) {
    last_error() = e.msg;
    return e.code;
  }
}

extern "C" int h2_tune_save(const char* path) {
  try {
    tune_save(path ? path : "");
    return H2_OK;
  } catch (const Error& e) {
    last_error() = e.msg;
    return e.code;
  }
}

extern "C" int h2_tune_report(char* buf, int64_t len) {
  try {
    if (!buf || len < 1) fail(H2_EINVAL, "null or empty buffer");
    const std::string r = tune_report();
    if (int64_t(r.size()) >= len) fail(H2_EINVAL, "buffer too small for the tuning report");
    std::memcpy(buf, r.c_str(), r.size() + 1);
    return H2_OK;
  } catch (const Error& e) {
    last_error() = e.msg;
    return e.code;
  }
}
