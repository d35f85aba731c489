// Tuning table (see tune.h): built-in defaults, a JSON cache keyed by GPU
// architecture, and the record of which entries the planned work used.
#include "tune.h"

#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <atomic>
#include <mutex>
#include <sstream>

#include "h2_internal.h"
#include "h2sp.h"
#include "kernels.h"

namespace h2 {

namespace {

std::mutex g_mu;
std::map<std::string, int64_t> g_table;  // entries that replace a default
std::map<std::string, int64_t> g_used_val;
std::string g_source = "defaults";
bool g_loaded = false;
std::atomic<int64_t> g_generation{0};

const char* role_name(int role) {
  switch (role) {
    case ROLE_FACTOR: return "factor";
    case ROLE_SOLVE: return "solve";
    case ROLE_MATVEC: return "matvec";
    default: return "transform";
  }
}

// Knobs and their accepted ranges.
struct Knob {
  const char* key;
  int64_t lo, hi;
};
constexpr Knob kKnobs[] = {
    {"schur.split_k", 16, int64_t(1) << 30},
    {"schur.key_z", 0, 1},
    {"schur.order_min", 1, int64_t(1) << 40},
    {"schur.split_big", 0, 1},
    {"solve.split_k", 16, int64_t(1) << 30},
    {"solve.transpose", 0, 1},
};

// Parses "gemm.<f32|f64>.<role>.a<am>b<bm>.m<bucket>"; false if malformed.
bool parse_gemm_key(const std::string& k, int* prec, int* role, int* am, int* bm, int* bucket) {
  char p[8] = {0}, r[16] = {0};
  int a = -1, b = -1, m = -1;
  if (std::sscanf(k.c_str(), "gemm.%3[f0-9].%15[a-z].a%db%d.m%d", p, r, &a, &b, &m) != 5) return false;
  const std::string ps(p), rs(r);
  if (ps != "f32" && ps != "f64") return false;
  int ro = -1;
  for (int i = 0; i < 4; ++i)
    if (rs == role_name(i)) ro = i;
  if (ro < 0 || a < 0 || a > 2 || b < 0 || b > 2 || m < 0 || m > 3) return false;
  if (gemm_key(ps == "f32" ? 1 : 0, ro, a, b, m) != k) return false;
  *prec = ps == "f32" ? 1 : 0;
  *role = ro;
  *am = a;
  *bm = b;
  *bucket = m;
  return true;
}

void check_entry(const std::string& key, int64_t value) {
  int prec, role, am, bm, bucket;
  if (parse_gemm_key(key, &prec, &role, &am, &bm, &bucket)) {
    if (!gemm_layout_supported(role, am, bm)) fail(H2_EINVAL, "tuning: no GEMM kernel for " + key);
    if (value < 0 || value >= kGemmVariants || gemm_shape(prec, role, am, bm, int(value)) == 0)
      fail(H2_EINVAL, "tuning: variant " + std::to_string(value) + " of " + key + " is not built");
    return;
  }
  for (const Knob& k : kKnobs)
    if (key == k.key) {
      if (value < k.lo || value > k.hi) fail(H2_EINVAL, "tuning: " + key + " out of range");
      return;
    }
  fail(H2_EINVAL, "tuning: unknown key " + key);
}

// ---- minimal JSON: an object of architecture names, each an object of
// integer entries.
struct Parser {
  const std::string& s;
  size_t i = 0;
  void ws() {
    while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) ++i;
  }
  void expect(char c) {
    ws();
    if (i >= s.size() || s[i] != c) fail(H2_EINVAL, std::string("tuning file: expected '") + c + "'");
    ++i;
  }
  bool peek(char c) {
    ws();
    return i < s.size() && s[i] == c;
  }
  std::string str() {
    expect('"');
    std::string out;
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\') fail(H2_EINVAL, "tuning file: escapes are not supported");
      out += s[i++];
    }
    expect('"');
    return out;
  }
  int64_t integer() {
    ws();
    size_t j = i;
    if (j < s.size() && s[j] == '-') ++j;
    while (j < s.size() && std::isdigit(static_cast<unsigned char>(s[j]))) ++j;
    if (j == i) fail(H2_EINVAL, "tuning file: expected an integer");
    const int64_t v = std::strtoll(s.c_str() + i, nullptr, 10);
    i = j;
    return v;
  }
  std::map<std::string, int64_t> entries() {
    std::map<std::string, int64_t> out;
    expect('{');
    if (peek('}')) {
      ++i;
      return out;
    }
    for (;;) {
      const std::string k = str();
      expect(':');
      out[k] = integer();
      if (peek(',')) {
        ++i;
        continue;
      }
      expect('}');
      return out;
    }
  }
  std::map<std::string, std::map<std::string, int64_t>> file() {
    std::map<std::string, std::map<std::string, int64_t>> out;
    expect('{');
    if (peek('}')) {
      ++i;
      return out;
    }
    for (;;) {
      const std::string arch = str();
      expect(':');
      out[arch] = entries();
      if (peek(',')) {
        ++i;
        continue;
      }
      expect('}');
      return out;
    }
  }
};

std::map<std::string, std::map<std::string, int64_t>> read_file(const std::string& path, bool must_exist) {
  std::ifstream f(path);
  if (!f) {
    if (must_exist) fail(H2_EINVAL, "tuning file not readable: " + path);
    return {};
  }
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  Parser p{text};
  auto out = p.file();
  p.ws();
  if (p.i != text.size()) fail(H2_EINVAL, "tuning file: trailing characters in " + path);
  return out;
}

std::string default_path() {
  if (const char* e = std::getenv("H2SP_TUNE_FILE")) return e;
  Dl_info info{};
  if (dladdr(reinterpret_cast<void*>(&default_path), &info) && info.dli_fname) {
    std::string so(info.dli_fname);
    const size_t slash = so.rfind('/');
    return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/tune.json";
  }
  return "tune.json";
}

// Caller holds g_mu.
void load_locked(const std::string& path, bool must_exist) {
  auto all = read_file(path, must_exist);
  const std::string arch = device_arch();
  auto it = all.find(arch);
  std::map<std::string, int64_t> table;
  if (it != all.end()) {
    for (const auto& kv : it->second) check_entry(kv.first, kv.second);
    table = it->second;
  }
  g_table.swap(table);
  g_source = it != all.end() ? path : "defaults";
  g_loaded = true;
  ++g_generation;
}

// A missing default cache means the defaults; a cache that is there but
// malformed, or names an entry that is not built, fails every call that plans.
void ensure_loaded_locked() {
  if (!g_loaded) load_locked(default_path(), std::getenv("H2SP_TUNE_FILE") != nullptr);
}

int64_t lookup_locked(const std::string& key, int64_t def) {
  ensure_loaded_locked();
  auto it = g_table.find(key);
  const int64_t v = it != g_table.end() ? it->second : def;
  g_used_val[key] = v;
  return v;
}

}  // namespace

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a(prop.gcnArchName);
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

int gemm_row_bucket(int max_m) { return max_m <= 16 ? 0 : max_m <= 32 ? 1 : max_m <= 64 ? 2 : 3; }

std::string gemm_key(int prec, int role, int am, int bm, int bucket) {
  char buf[64];
  std::snprintf(buf, sizeof buf, "gemm.%s.%s.a%db%d.m%d", prec ? "f32" : "f64", role_name(role), am, bm, bucket);
  return buf;
}

int tune_gemm_variant(int prec, int role, int am, int bm, int bucket) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int v = int(lookup_locked(gemm_key(prec, role, am, bm, bucket), 0));
  return gemm_shape(prec, role, am, bm, v) != 0 ? v : 0;
}

int64_t tune_knob(const char* key, int64_t def) {
  std::lock_guard<std::mutex> lk(g_mu);
  return lookup_locked(key, def);
}

void tune_set(const std::string& key, int64_t value) {
  check_entry(key, value);
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded_locked();
  g_table[key] = value;
  g_source = "set";
  ++g_generation;
}

bool tune_get(const std::string& key, int64_t* value) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded_locked();
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  *value = it->second;
  return true;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  g_used_val.clear();
  g_source = "defaults";
  g_loaded = true;
  ++g_generation;
}

void tune_load(const std::string& path) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked(path.empty() ? default_path() : path, true);
  g_used_val.clear();
}

void tune_save(const std::string& path) {
  std::lock_guard<std::mutex> lk(g_mu);
  ensure_loaded_locked();
  const std::string p = path.empty() ? default_path() : path;
  auto all = read_file(p, false);
  all[device_arch()] = g_table;
  std::ofstream f(p);
  if (!f) fail(H2_EINVAL, "tuning file not writable: " + p);
  f << "{\n";
  size_t a = 0;
  for (const auto& arch : all) {
    f << "  \"" << arch.first << "\": {";
    size_t e = 0;
    for (const auto& kv : arch.second)
      f << (e++ ? ",\n    " : "\n    ") << "\"" << kv.first << "\": " << kv.second;
    f << (arch.second.empty() ? "}" : "\n  }") << (++a < all.size() ? ",\n" : "\n");
  }
  f << "}\n";
  if (!f) fail(H2_EINVAL, "tuning file write failed: " + p);
}

int64_t tune_generation() { return g_generation.load(); }

void tune_reset_used() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_used_val.clear();
}

std::string tune_report() {
  std::lock_guard<std::mutex> lk(g_mu);
  std::ostringstream o;
  o << "{\"arch\": \"" << device_arch() << "\", \"source\": \"" << g_source << "\", \"used\": {";
  size_t e = 0;
  for (const auto& kv : g_used_val) o << (e++ ? ", " : "") << "\"" << kv.first << "\": " << kv.second;
  o << "}}";
  return o.str();
}

}  // namespace h2
