// Tuning table of the library: the output tile shape of each GEMM role and
// operand layout (per precision and bucket of item rows) and the knobs of the
// Schur update's work lists.  Defaults are the built-in values; a JSON cache,
// one object per GPU architecture, replaces them (loaded once per process,
// from H2SP_TUNE_FILE or tune.json beside the library); the autotuner writes
// it.  Every entry changes the speed only: results are the same bit for bit.
#pragma once

#include <cstdint>
#include <string>

namespace h2 {

// Row bucket of a GEMM batch by its largest item row count: <= 16, <= 32,
// <= 64, more.
int gemm_row_bucket(int max_m);
// Key of a GEMM entry, e.g. "gemm.f32.solve.a1b0.m3".
std::string gemm_key(int prec, int role, int am, int bm, int bucket);
// The tile variant a batch of this kind runs (recorded as used).
int tune_gemm_variant(int prec, int role, int am, int bm, int bucket);
// An integer knob ("schur.split_k", "schur.key_z", "schur.order_min"),
// recorded as used.
int64_t tune_knob(const char* key, int64_t def);

// Entry points behind the C-ABI (codes of h2sp.h; messages through fail()).
void tune_set(const std::string& key, int64_t value);
bool tune_get(const std::string& key, int64_t* value);
void tune_clear();
void tune_load(const std::string& path);
void tune_save(const std::string& path);
std::string tune_report();  // JSON: arch, source, entries used since the last clear
std::string device_arch();  // "gfx950" (the part of gcnArchName before ':')
// Changes whenever an entry may have changed; work lists planned under an
// older generation are planned again before they run.
int64_t tune_generation();
// Forgets which entries were used (the next tune_report lists only later use).
void tune_reset_used();

}  // namespace h2
