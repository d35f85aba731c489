// Sparsification sweep (Section 2 "Compression at all levels", Algorithm 1 as
// built from H^2 coefficients in Section 4.2-4.3), planned on the host and run
// level by level on the device.
//
// Level k, for every cluster t on it (n_t active rows, k_t kept, m_t = n_t - k_t):
//  1. B_t = R_t (leaf) or [R^_c1 T_c1; R^_c2 T_c2]; Householder QR B_t = Q_t [R^_t; 0]
//     with explicit square Q_t (FP64, batched);
//  2. every close pair (t, s) in N_k, t <= s: X = Q_t^T C_k(t,s) Q_s with
//     C_0 = kernel block (generated in registers), C_k = block assembled at level
//     k-1; X's four quadrants go to S (non-basis x non-basis), to the father's
//     close block (basis x basis), and to the row strips of the finalised rows;
//  3. every interaction pair (a, b) in I_k: R^_a D_ab R^_b^T into the father's
//     close block (D_ab = P_a K(nodes_a, nodes_b) P_b^T);
//  4. every strip G(tau, p) of rows finalised below level k: Y = G Q_p; the
//     non-basis columns are the off-level block S(tau, p) (Section 3), the basis
//     columns travel on to p's father.
// S keeps its upper block triangle (S symmetric, Proposition 2.1): lower-level
// rows first, clusters left to right.
#include <algorithm>
#include <cstdio>
#include <chrono>
#include <cstring>
#include <memory>
#include <parallel/algorithm>
#include <string>

#include "sparse.h"

namespace h2 {

namespace {

constexpr i64 kTmpChunkEntries = i64(1) << 26;  // GEMM temporaries per chunk

inline i64 key(i64 a, i64 b, i64 ncl) { return a * ncl + b; }

// Slot table of one level: open addressing with linear probing over
// non-negative keys, power-of-two capacity, no deletion.  (A node-based map
// of a few million entries costs more to fill, probe and free than the whole
// sweep's planning otherwise.)
class SlotMap {
 public:
  void reserve(size_t n) {
    size_t cap = 16;
    while (cap < 2 * n) cap <<= 1;
    if (cap > keys_.size()) rehash(cap);
  }
  // inserts (k, v) unless k is present; returns whether it inserted
  bool insert(i64 k, i64 v) {
    if (2 * (size_ + 1) > keys_.size()) rehash(std::max<size_t>(16, 2 * keys_.size()));
    size_t h = hash(k) & (keys_.size() - 1);
    while (keys_[h] >= 0) {
      if (keys_[h] == k) return false;
      h = (h + 1) & (keys_.size() - 1);
    }
    keys_[h] = k;
    vals_[h] = v;
    ++size_;
    return true;
  }
  // inserts a key known to be absent, from several threads at once; the table
  // must have been reserved for every key inserted this way (no growth)
  void insert_distinct_concurrent(i64 k, i64 v) {
    const size_t mask = keys_.size() - 1;
    size_t h = hash(k) & mask;
    while (true) {
      i64 expect = -1;
      if (__atomic_compare_exchange_n(&keys_[h], &expect, k, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) break;
      h = (h + 1) & mask;
    }
    vals_[h] = v;
  }
  void count_inserted(size_t n) { size_ += n; }
  i64 at(i64 k) const {
    if (!keys_.empty()) {
      size_t h = hash(k) & (keys_.size() - 1);
      while (keys_[h] >= 0) {
        if (keys_[h] == k) return vals_[h];
        h = (h + 1) & (keys_.size() - 1);
      }
    }
    fail(H2_EINVAL, "internal: missing slot");
  }

 private:
  // 64-bit finaliser of MurmurHash3 (public domain)
  static uint64_t hash(i64 k) {
    uint64_t x = uint64_t(k);
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
  }
  void rehash(size_t cap) {
    std::vector<i64> ok, ov;
    ok.swap(keys_);
    ov.swap(vals_);
    keys_.assign(cap, -1);
    vals_.resize(cap);
    size_ = 0;
    for (size_t i = 0; i < ok.size(); ++i)
      if (ok[i] >= 0) insert(ok[i], ov[i]);
  }
  std::vector<i64> keys_, vals_;
  size_t size_ = 0;
};

struct SymStrip {
  int32_t tau, p;
  i64 slot;
};

}  // namespace

// symbolic: sizes, elimination order and S pattern only, on the host (no
// device memory, no upload of the H^2 coefficients); such a handle is not
// sparsified and serves only to count (h2_plan_report)
static h2_sparse* plan(h2_matrix* H, int precision, bool upload, bool symbolic = false) {
  TraceTimer tt("sparsify-plan");
  if (!symbolic) H->upload_all();
  auto spp = std::make_unique<h2_sparse>();
  h2_sparse& sp = *spp;
  const Tree& tr = H->tree;
  const int L = tr.depth, dim = tr.dim, P = H->P;
  const i64 ncl = tr.ncl();
  sp.H = H;
  sp.precision = precision;
  sp.ncl = ncl;
  sp.elem = precision == H2_MIXED ? sizeof(float) : sizeof(double);

  // ---- sizes n_t, k_t, m_t
  sp.n_act.assign(ncl, 0);
  sp.kept.assign(ncl, 0);
  for (int k = 0; k <= L; ++k) {
    const i64 f = tr.first_at_level(k), cnt = tr.count_at_level(k);
    for (i64 c = f; c < f + cnt; ++c) {
      sp.n_act[c] = (k == 0) ? tr.size[c] : sp.kept[2 * c + 1] + sp.kept[2 * c + 2];
      sp.kept[c] = H->ff[c] ? std::min<i64>(sp.n_act[c], H->rank[c]) : 0;
      if (sp.n_act[c] > 128) fail(H2_EUNSUPPORTED, "active cluster size above 128");
      if (H->ff[c] && H->rank[c] > 64) fail(H2_EUNSUPPORTED, "rank above 64");
    }
  }
  sp.nonbasis.resize(ncl);
  for (i64 c = 0; c < ncl; ++c) sp.nonbasis[c] = sp.n_act[c] - sp.kept[c];
  // ---- S order (level 0 first, left to right)
  sp.order.clear();
  for (int k = 0; k <= L; ++k)
    for (i64 c = tr.first_at_level(k); c < tr.first_at_level(k) + tr.count_at_level(k); ++c)
      sp.order.push_back(c);
  sp.spos.assign(ncl, 0);
  sp.soff.assign(ncl, 0);
  i64 pos = 0;
  for (i64 i = 0; i < ncl; ++i) {
    sp.spos[sp.order[i]] = i;
    sp.soff[sp.order[i]] = pos;
    pos += sp.nonbasis[sp.order[i]];
  }
  if (pos != tr.n) fail(H2_EINVAL, "internal: non-basis rows do not add up to n");
  const auto& n_act = sp.n_act;
  const auto& kept = sp.kept;
  const auto& mb = sp.nonbasis;
  auto son_off = [&](i64 c) -> i64 { return (c % 2 == 1) ? 0 : kept[c - 1]; };

  // ---- elimination order: per level, greedy colouring of the close graph
  // among clusters with non-basis rows, then (colour, cluster)
  sp.colour.assign(ncl, -1);
  sp.eorder.clear();
  sp.epos.assign(ncl, 0);
  for (int k = 0; k <= L; ++k) {
    const i64 f = tr.first_at_level(k), cnt = tr.count_at_level(k);
    std::vector<std::vector<i64>> earlier(cnt);
    for (const Pair& pr : H->bt.near[k])
      if (pr.s < pr.t && mb[pr.t] > 0 && mb[pr.s] > 0) earlier[pr.t - f].push_back(pr.s);
    std::vector<char> taken;
    for (i64 c = f; c < f + cnt; ++c) {
      if (mb[c] == 0) continue;
      taken.assign(earlier[c - f].size() + 1, 0);
      for (i64 s : earlier[c - f])
        if (sp.colour[s] < int(taken.size())) taken[sp.colour[s]] = 1;
      int col = 0;
      while (taken[col]) ++col;
      sp.colour[c] = col;
    }
    std::vector<i64> lv;
    for (i64 c = f; c < f + cnt; ++c)
      if (mb[c] > 0) lv.push_back(c);
    std::stable_sort(lv.begin(), lv.end(), [&](i64 a, i64 b) { return sp.colour[a] < sp.colour[b]; });
    for (i64 c = f; c < f + cnt; ++c)
      if (mb[c] == 0) lv.push_back(c);
    sp.eorder.insert(sp.eorder.end(), lv.begin(), lv.end());
  }
  for (i64 i = 0; i < ncl; ++i) sp.epos[sp.eorder[i]] = i;
  const auto& epos = sp.epos;

  tt.lap("order");
  // ---- symbolic sweep: strips, close/coupling lists, C slots, S blocks
  std::vector<std::vector<Pair>> closeL(L + 1), coupL(L + 1);
  std::vector<std::vector<SymStrip>> stripL(L + 2);
  std::vector<SlotMap> cslot(L + 2), gslot(L + 2);
  std::vector<i64> csize(L + 2, 0), gsize(L + 2, 0);
  std::vector<std::pair<i64, i64>> blocks;  // (t, s) with epos(t) <= epos(s)
  double sym_ms[3] = {0, 0, 0};             // traced split of the sweep
  // Per level, in parallel: every strip of the level and every close pair
  // writes its S block and its candidate strips of the next level at fixed
  // positions (strips first, then pairs, in order); the candidates are then
  // made distinct keeping each key's first occurrence, and the next level's
  // strips take their slots in that order (the layout a sequential sweep
  // gives).
  struct Cand {
    i64 key;
    int32_t tau, p;
  };
  for (int k = 0; k <= L; ++k) {
    const auto c0 = std::chrono::steady_clock::now();
    const std::vector<SymStrip>& sk = stripL[k];
    const std::vector<Pair>& nk = H->bt.near[k];
    const long ns = long(sk.size()), nn = long(nk.size());
    std::vector<Cand> cand(size_t(ns + 2 * nn), Cand{-1, 0, 0});
    std::vector<std::pair<i64, i64>> blk(size_t(ns + nn), std::make_pair(i64(-1), i64(-1)));
    std::vector<char> is_close(size_t(nn), 0);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < ns; ++i) {
      const SymStrip& g = sk[i];
      if (mb[g.p] > 0) blk[i] = {g.tau, g.p};
      if (kept[g.p] > 0 && g.p > 0) {
        const i64 f = (g.p - 1) / 2;
        cand[i] = {key(g.tau, f, ncl), g.tau, int32_t(f)};
      }
    }
#pragma omp parallel for schedule(static)
    for (long j = 0; j < nn; ++j) {
      const i64 t = nk[j].t, s = nk[j].s;
      if (t > s || n_act[t] == 0 || n_act[s] == 0) continue;
      is_close[j] = 1;
      if (mb[t] > 0 && mb[s] > 0) blk[ns + j] = epos[t] <= epos[s] ? std::make_pair(t, s) : std::make_pair(s, t);
      if (k < L) {
        if (mb[t] > 0 && kept[s] > 0) cand[ns + 2 * j] = {key(t, (s - 1) / 2, ncl), int32_t(t), int32_t((s - 1) / 2)};
        if (t != s && mb[s] > 0 && kept[t] > 0)
          cand[ns + 2 * j + 1] = {key(s, (t - 1) / 2, ncl), int32_t(s), int32_t((t - 1) / 2)};
      }
    }
    for (long j = 0; j < nn; ++j)
      if (is_close[j]) closeL[k].push_back(nk[j]);
    for (const auto& b : blk)
      if (b.first >= 0) blocks.push_back(b);
    const auto c1 = std::chrono::steady_clock::now();
    // distinct candidates, first occurrence first
    std::vector<std::pair<i64, i64>> kv;  // (key, position)
    kv.reserve(cand.size());
    for (size_t q = 0; q < cand.size(); ++q)
      if (cand[q].key >= 0) kv.push_back({cand[q].key, i64(q)});
    sort_range(kv.begin(), kv.end());
    std::vector<i64> first;
    first.reserve(kv.size());
    for (size_t q = 0; q < kv.size(); ++q)
      if (q == 0 || kv[q].first != kv[q - 1].first) first.push_back(kv[q].second);
    sort_range(first.begin(), first.end());
    std::vector<SymStrip>& nxt = stripL[k + 1];
    nxt.reserve(first.size());
    for (i64 q : first) {
      const Cand& c = cand[size_t(q)];
      nxt.push_back({c.tau, c.p, gsize[k + 1]});
      gsize[k + 1] += mb[c.tau] * n_act[c.p];
    }
    gslot[k + 1].reserve(nxt.size());
#pragma omp parallel for schedule(static)
    for (long q = 0; q < long(nxt.size()); ++q)
      gslot[k + 1].insert_distinct_concurrent(key(nxt[q].tau, nxt[q].p, ncl), nxt[q].slot);
    gslot[k + 1].count_inserted(nxt.size());
    const auto c2 = std::chrono::steady_clock::now();
    for (const Pair& pr : H->bt.far[k])
      if (pr.t < pr.s) coupL[k].push_back(pr);
    if (k < L) {
      cslot[k + 1].reserve(H->bt.near[k + 1].size());
      for (const Pair& pr : H->bt.near[k + 1]) {
        if (pr.t > pr.s || n_act[pr.t] == 0 || n_act[pr.s] == 0) continue;
        cslot[k + 1].insert(key(pr.t, pr.s, ncl), csize[k + 1]);
        csize[k + 1] += n_act[pr.t] * n_act[pr.s];
      }
    }
    const auto c3 = std::chrono::steady_clock::now();
    sym_ms[0] += std::chrono::duration<double, std::milli>(c1 - c0).count();
    sym_ms[1] += std::chrono::duration<double, std::milli>(c2 - c1).count();
    sym_ms[2] += std::chrono::duration<double, std::milli>(c3 - c2).count();
  }
  if (trace_enabled())
    std::fprintf(stderr, "[h2sp] sparsify-plan symbolic: blocks and candidates %.1f ms, distinct strips %.1f ms, far pairs and slots %.1f ms; "
                 "%zu blocks, %zu strips\n", sym_ms[0], sym_ms[1], sym_ms[2], blocks.size(),
                 [&] { size_t n = 0; for (auto& v : stripL) n += v.size(); return n; }());
  tt.lap("symbolic");
  // ---- upper block pattern in the elimination order: blocks as
  // (row position, column position) keys, sorted in parallel
  std::vector<uint64_t> bkeys(blocks.size());
  for (size_t b = 0; b < blocks.size(); ++b)
    bkeys[b] = (uint64_t(epos[blocks[b].first]) << 32) | uint64_t(epos[blocks[b].second]);
  std::vector<std::pair<i64, i64>>().swap(blocks);
  sort_range(bkeys.begin(), bkeys.end());
  if (std::adjacent_find(bkeys.begin(), bkeys.end()) != bkeys.end())
    fail(H2_EINVAL, "internal: duplicate S block");
  sp.rowptr.assign(ncl + 1, 0);
  sp.colidx.resize(bkeys.size());
  sp.blk_off.resize(bkeys.size());
  i64 ent = 0;
  for (size_t b = 0; b < bkeys.size(); ++b) {
    const i64 t = sp.eorder[i64(bkeys[b] >> 32)], s = sp.eorder[i64(bkeys[b] & 0xffffffffu)];
    sp.rowptr[epos[t] + 1]++;
    sp.colidx[b] = s;
    sp.blk_off[b] = ent;
    ent += mb[t] * mb[s];
  }
  std::vector<uint64_t>().swap(bkeys);
  tt.lap("pattern");
  for (i64 i = 0; i < ncl; ++i) sp.rowptr[i + 1] += sp.rowptr[i];
  sp.s_entries = ent;

  // ---- arenas (level-contiguous so that one cast covers a level)
  sp.q_off.assign(ncl, -1);
  sp.b_off.assign(ncl, -1);
  sp.rhat_off.assign(ncl, -1);
  sp.w_off.assign(ncl, -1);
  std::vector<i64> qlev(L + 2, 0), wlev(L + 2, 0);
  i64 qs = 0, bs = 0, rs = 0, ws = 0;
  for (int k = 0; k <= L; ++k) {
    qlev[k] = qs;
    wlev[k] = H->identity_proj ? rs : ws;
    for (i64 c = tr.first_at_level(k); c < tr.first_at_level(k) + tr.count_at_level(k); ++c) {
      if (n_act[c] == 0) continue;
      sp.q_off[c] = qs;
      qs += n_act[c] * n_act[c];
      if (kept[c] > 0) {
        if (k > 0) {
          sp.b_off[c] = bs;
          bs += n_act[c] * H->rank[c];
        }
        sp.rhat_off[c] = rs;
        rs += kept[c] * H->rank[c];
        if (!H->identity_proj) {
          sp.w_off[c] = ws;
          ws += kept[c] * P;
        }
      }
    }
    qlev[k + 1] = qs;
    wlev[k + 1] = H->identity_proj ? rs : ws;
  }
  if (symbolic) {
    sp.q_entries = qs;
    return spp.release();
  }
  const bool mixed = precision == H2_MIXED;
  const size_t el = sp.elem;
  sp.dQ.reset(8 * std::max<i64>(qs, 1));
  sp.dB.reset(8 * std::max<i64>(bs, 1));
  sp.dRhat.reset(8 * std::max<i64>(rs, 1));
  if (!H->identity_proj) sp.dW.reset(8 * std::max<i64>(ws, 1));
  if (mixed) {
    sp.dQt.reset(4 * std::max<i64>(qs, 1));
    sp.dWt.reset(4 * std::max<i64>(H->identity_proj ? rs : ws, 1));
  }
  sp.dS.reset(el * std::max<i64>(ent, 1));
  i64 cmax[2] = {1, 1}, gmax[2] = {1, 1};
  for (int k = 0; k <= L + 1; ++k) {
    cmax[k % 2] = std::max(cmax[k % 2], csize[k]);
    gmax[k % 2] = std::max(gmax[k % 2], gsize[k]);
  }
  for (int side = 0; side < 2; ++side) {
    sp.dC[side].reset(el * cmax[side]);
    sp.dG[side].reset(el * gmax[side]);
  }
  sp.dTmp.reset(el * kTmpChunkEntries);

  tt.lap("arenas");
  // ---- per-level work lists with device pointers
  const double* X = H->d_x.as<double>();
  const double* nodes = H->d_nodes.as<double>();
  char* S = static_cast<char*>(sp.dS.ptr);
  char* Qt = mixed ? static_cast<char*>(sp.dQt.ptr) : static_cast<char*>(sp.dQ.ptr);
  char* Wt = mixed ? static_cast<char*>(sp.dWt.ptr)
                   : static_cast<char*>(H->identity_proj ? sp.dRhat.ptr : sp.dW.ptr);
  const std::vector<i64>& wtoff = H->identity_proj ? sp.rhat_off : sp.w_off;
  char* tmp = static_cast<char*>(sp.dTmp.ptr);
  double* dQ = sp.dQ.as<double>();
  double* dB = sp.dB.as<double>();
  double* dR = sp.dRhat.as<double>();
  double* dW = sp.dW.as<double>();
  const double* basis = H->d_basis.as<double>();
  const double* transfer = H->d_transfer.as<double>();
  const double* proj = H->d_proj.as<double>();
  std::vector<PlanCounts> lpc(L + 1);
  sp.levels.resize(L + 1);
  auto blk_ptr = [&](i64 t, i64 s) -> void* {
    const i64 b = sp.block_of(t, s);
    if (b < 0) fail(H2_EINVAL, "internal: missing S block");
    return S + el * sp.blk_off[b];
  };
  // destination of S(t, s) as seen from the pair's orientation: stored as is,
  // or as the transposed block (s, t) when s comes first in elimination order
  auto set_s_out = [&](GemmItem& it, int q, i64 t, i64 s) {
    if (epos[t] <= epos[s]) GemmBatch::set_out(it, q, blk_ptr(t, s), mb[t], false);
    else GemmBatch::set_out(it, q, blk_ptr(s, t), mb[s], true);
  };
  // Levels are independent once slots and offsets are fixed, and so are the
  // pieces of a level: its QR and stacking items, runs of its strips, and the
  // chunks of its close and coupling pairs (chunk boundaries fixed first, by
  // the temporary space each pair takes).  Strip runs are appended in order
  // afterwards.
  std::string first_error;
  int first_code = 0;
  auto guarded = [&](auto&& body) {
    try {
      body();
    } catch (const Error& e) {
#pragma omp critical(h2_plan_error)
      if (!first_code) { first_code = e.code; first_error = e.msg; }
    } catch (const std::exception& e) {
#pragma omp critical(h2_plan_error)
      if (!first_code) { first_code = H2_EINVAL; first_error = e.what(); }
    }
  };
  auto chunk_starts = [](i64 count, auto&& size_of) {
    std::vector<i64> st;
    i64 used = kTmpChunkEntries;
    for (i64 i = 0; i < count; ++i) {
      const i64 sz = size_of(i);
      if (used + sz > kTmpChunkEntries) {
        st.push_back(i);
        used = 0;
      }
      used += sz;
    }
    st.push_back(count);
    return st;
  };
  constexpr i64 kStripRun = 32768;
  std::vector<std::vector<GemmBatch>> strip_runs(L + 1);
  std::vector<std::vector<i64>> close_cut(L + 1), coup_cut(L + 1);
  std::vector<std::vector<PlanCounts>> close_pc(L + 1), coup_pc(L + 1);
  for (int k = 0; k <= L; ++k) {
    close_cut[k] = chunk_starts(i64(closeL[k].size()),
                                [&](i64 i) { return n_act[closeL[k][i].t] * n_act[closeL[k][i].s]; });
    coup_cut[k] = chunk_starts(i64(coupL[k].size()), [&](i64 i) { return i64(P) * kept[coupL[k][i].s]; });
    const size_t ncl_chunks = close_cut[k].size() - 1, ncp_chunks = coup_cut[k].size() - 1;
    sp.levels[k].close1.resize(ncl_chunks);
    sp.levels[k].close2.resize(ncl_chunks);
    sp.levels[k].coup1.resize(ncp_chunks);
    sp.levels[k].coup2.resize(ncp_chunks);
    close_pc[k].resize(ncl_chunks);
    coup_pc[k].resize(ncp_chunks);
    strip_runs[k].resize((stripL[k].size() + kStripRun - 1) / kStripRun);
  }
  // one work unit per piece; units of every level in one worksharing loop
  // (no OpenMP tasks: this also runs on the batched path's pool threads,
  // where libomp's task allocator is not safe)
  struct Unit {
    int kind, k;  // kind 0: QR and stacking items, 1: strip run, 2: close chunk, 3: coupling chunk
    i64 idx;
  };
  std::vector<Unit> units;
  for (int k = 0; k <= L; ++k) {
    SweepLevel& lv = sp.levels[k];
    lv.gnext_side = (k + 1) % 2;
    lv.gnext_entries = (k < L) ? gsize[k + 1] : 0;
    units.push_back({0, k, 0});
    for (size_t run = 0; run < strip_runs[k].size(); ++run) units.push_back({1, k, i64(run)});
    for (size_t ch = 0; ch + 1 < close_cut[k].size(); ++ch) units.push_back({2, k, i64(ch)});
    for (size_t ch = 0; ch + 1 < coup_cut[k].size(); ++ch) units.push_back({3, k, i64(ch)});
  }
  auto qr_unit = [&](int k) {
    PlanCounts& pc = lpc[k];
    SweepLevel& lv = sp.levels[k];
    // 1. QR items
    std::vector<QrItem> qi;
    for (i64 c = tr.first_at_level(k); c < tr.first_at_level(k) + tr.count_at_level(k); ++c) {
      if (n_act[c] == 0) continue;
      QrItem it{};
      it.n = int32_t(n_act[c]);
      it.k = int32_t(kept[c]);
      it.r = kept[c] > 0 ? H->rank[c] : 0;
      it.Q = dQ + sp.q_off[c];
      if (kept[c] > 0) {
        it.B = (k == 0) ? basis + H->basis_off[c] : dB + sp.b_off[c];
        it.Rhat = dR + sp.rhat_off[c];
        const double n = it.n, r = it.r, q = std::min(it.n, it.r);
        pc.flops_qr += 2 * n * r * r - 2.0 / 3 * r * r * r + 4 * n * n * q - 4 * n * q * q + 4.0 / 3 * q * q * q;
        pc.bytes_qr += 8 * (n * r + n * n + double(it.k) * r);
      } else {
        pc.bytes_qr += 8.0 * it.n * it.n;
      }
      qi.push_back(it);
    }
    lv.qr.count = int(qi.size());
    lv.qr.items = std::move(qi);
    lv.qr.q_begin = qlev[k];
    lv.qr.q_end = qlev[k + 1];
    lv.qr.w_begin = wlev[k];
    lv.qr.w_end = wlev[k + 1];
    // 2. stack into the father's B, and W = R^ P
    for (i64 c = tr.first_at_level(k); c < tr.first_at_level(k) + tr.count_at_level(k); ++c) {
      if (kept[c] == 0) continue;
      const int r = H->rank[c];
      if (c > 0 && kept[(c - 1) / 2] > 0) {
        const i64 f = (c - 1) / 2;
        const int rf = H->rank[f];
        GemmItem& it = lv.stack.item(int(kept[c]), rf, int(kept[c]), rf);
        GemmBatch::set_out(it, 0, dB + sp.b_off[f] + son_off(c), n_act[f], false);
        lv.stack.seg(dR + sp.rhat_off[c], int(kept[c]), false, transfer + H->transfer_off[c], r, false, r);
      }
      if (!H->identity_proj) {
        GemmItem& it = lv.wproj.item(int(kept[c]), P, int(kept[c]), P);
        GemmBatch::set_out(it, 0, dW + sp.w_off[c], kept[c], false);
        lv.wproj.seg(dR + sp.rhat_off[c], int(kept[c]), false, proj + H->proj_off[c], r, false, r);
      }
    }
    pc.flops_misc += lv.stack.flops + lv.wproj.flops;
  };
  // 3. strips: G(tau, p) Q_p, in runs
  auto strip_unit = [&](int k, size_t run) {
    char* Gcur = static_cast<char*>(sp.dG[k % 2].ptr);
    char* Gnext = static_cast<char*>(sp.dG[(k + 1) % 2].ptr);
    GemmBatch& g = strip_runs[k][run];
    const size_t b0 = run * kStripRun, b1 = std::min(stripL[k].size(), b0 + kStripRun);
    for (size_t q = b0; q < b1; ++q) {
      const SymStrip& gs = stripL[k][q];
      const i64 tau = gs.tau, p = gs.p;
      GemmItem& it = g.item(int(mb[tau]), int(n_act[p]), 0, int(kept[p]));
      if (mb[p] > 0) GemmBatch::set_out(it, 3, blk_ptr(tau, p), mb[tau], false);
      if (kept[p] > 0 && p > 0) {
        const i64 f = (p - 1) / 2;
        const i64 slot = gslot[k + 1].at(key(tau, f, ncl));
        GemmBatch::set_out(it, 2, Gnext + el * (slot + son_off(p) * mb[tau]), mb[tau], false);
      }
      g.seg(Gcur + el * gs.slot, int(mb[tau]), false, Qt + el * sp.q_off[p], int(n_act[p]), false,
            int(n_act[p]));
    }
  };
  // 4. close pairs, one unit per chunk of temporary space
  auto close_unit = [&](int k, size_t ch) {
    char* Ccur = static_cast<char*>(sp.dC[k % 2].ptr);
    char* Cnext = static_cast<char*>(sp.dC[(k + 1) % 2].ptr);
    char* Gnext = static_cast<char*>(sp.dG[(k + 1) % 2].ptr);
    SweepLevel& lv = sp.levels[k];
    GemmBatch& g1 = lv.close1[ch];
    GemmBatch& g2 = lv.close2[ch];
    i64 used = 0;
    for (i64 i = close_cut[k][ch]; i < close_cut[k][ch + 1]; ++i) {
      const Pair& pr = closeL[k][i];
      const i64 t = pr.t, s = pr.s, nt = n_act[t], ns = n_act[s];
      char* w = tmp + el * used;
      used += nt * ns;
      GemmItem& a = g1.item(int(nt), int(ns), int(nt), int(ns));
      GemmBatch::set_out(a, 0, w, nt, false);
      if (k == 0)
        g1.seg_gen(X + tr.start[t] * dim, X + tr.start[s] * dim, t == s, Qt + el * sp.q_off[s], int(ns), false,
                   int(ns));
      else
        g1.seg(Ccur + el * cslot[k].at(key(t, s, ncl)), int(nt), false, Qt + el * sp.q_off[s], int(ns), false,
               int(ns));
      GemmItem& b = g2.item(int(nt), int(ns), int(kept[t]), int(kept[s]));
      if (mb[t] > 0 && mb[s] > 0) set_s_out(b, 3, t, s);
      if (k < L) {
        const i64 pt = (t - 1) / 2, ps = (s - 1) / 2;
        if (kept[t] > 0 && kept[s] > 0) {
          char* cs = Cnext + el * cslot[k + 1].at(key(pt, ps, ncl));
          GemmBatch::set_out(b, 0, cs + el * (son_off(t) + son_off(s) * n_act[pt]), n_act[pt], false);
          if (pt == ps && t != s)
            GemmBatch::set_out(b, 4, cs + el * (son_off(s) + son_off(t) * n_act[pt]), n_act[pt], true);
        }
        if (mb[t] > 0 && kept[s] > 0) {
          const i64 slot = gslot[k + 1].at(key(t, ps, ncl));
          GemmBatch::set_out(b, 2, Gnext + el * (slot + son_off(s) * mb[t]), mb[t], false);
        }
        if (t != s && mb[s] > 0 && kept[t] > 0) {
          const i64 slot = gslot[k + 1].at(key(s, pt, ncl));
          GemmBatch::set_out(b, 1, Gnext + el * (slot + son_off(t) * mb[s]), mb[s], true);
        }
      }
      g2.seg(Qt + el * sp.q_off[t], int(nt), true, w, int(nt), false, int(nt));
    }
    close_pc[k][ch].flops_close = g1.flops + g2.flops;
  };
  // 5. couplings R^_a D_ab R^_b^T into the father's close block, per chunk
  auto coup_unit = [&](int k, size_t ch) {
    char* Cnext = static_cast<char*>(sp.dC[(k + 1) % 2].ptr);
    SweepLevel& lv = sp.levels[k];
    GemmBatch& g1 = lv.coup1[ch];
    GemmBatch& g2 = lv.coup2[ch];
    i64 used = 0;
    for (i64 i = coup_cut[k][ch]; i < coup_cut[k][ch + 1]; ++i) {
      const Pair& pr = coupL[k][i];
      const i64 a = pr.t, b = pr.s;
      const i64 ka = kept[a], kb = kept[b];
      if (ka == 0 || kb == 0) fail(H2_EINVAL, "internal: coupling of a cluster without kept rows");
      char* w = tmp + el * used;
      used += P * kb;
      GemmItem& i1 = g1.item(P, int(kb), P, int(kb));
      GemmBatch::set_out(i1, 0, w, P, false);
      g1.seg_gen(nodes + a * i64(P) * dim, nodes + b * i64(P) * dim, false, Wt + el * wtoff[b], int(kb), true, P);
      const i64 pa = (a - 1) / 2, pb = (b - 1) / 2;
      GemmItem& i2 = g2.item(int(ka), int(kb), int(ka), int(kb));
      char* cs = Cnext + el * cslot[k + 1].at(key(pa, pb, ncl));
      GemmBatch::set_out(i2, 0, cs + el * (son_off(a) + son_off(b) * n_act[pa]), n_act[pa], false);
      if (pa == pb)
        GemmBatch::set_out(i2, 4, cs + el * (son_off(b) + son_off(a) * n_act[pa]), n_act[pa], true);
      g2.seg(Wt + el * wtoff[a], int(ka), false, w, P, false, P);
    }
    coup_pc[k][ch].flops_coup = g1.flops + g2.flops;
  };
#pragma omp parallel for schedule(dynamic, 1)
  for (long u = 0; u < long(units.size()); ++u) {
    const Unit un = units[u];
    guarded([&] {
      switch (un.kind) {
        case 0: qr_unit(un.k); break;
        case 1: strip_unit(un.k, size_t(un.idx)); break;
        case 2: close_unit(un.k, size_t(un.idx)); break;
        default: coup_unit(un.k, size_t(un.idx)); break;
      }
    });
  }
  // strip runs appended in order (levels in parallel), per-chunk counts summed
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k <= L; ++k) {
    if (first_code) continue;
    guarded([&, k] {
      SweepLevel& lv = sp.levels[k];
      size_t ni = 0, ns = 0;
      for (const GemmBatch& g : strip_runs[k]) ni += g.items.size(), ns += g.segs.size();
      lv.strips.items.reserve(ni);
      lv.strips.segs.reserve(ns);
      for (GemmBatch& g : strip_runs[k]) lv.strips.append(g);
      lpc[k].flops_strip += lv.strips.flops;
      for (const PlanCounts& c : close_pc[k]) lpc[k].flops_close += c.flops_close;
      for (const PlanCounts& c : coup_pc[k]) lpc[k].flops_coup += c.flops_coup;
    });
  }
  if (first_code) fail(first_code, first_error);
  for (const PlanCounts& c : lpc) {
    sp.counts.flops_qr += c.flops_qr;
    sp.counts.flops_close += c.flops_close;
    sp.counts.flops_coup += c.flops_coup;
    sp.counts.flops_strip += c.flops_strip;
    sp.counts.flops_misc += c.flops_misc;
    sp.counts.bytes_qr += c.bytes_qr;
  }
  // ---- one device allocation for every work list of the sweep
  std::vector<GemmBatch*> all;
  std::vector<RawBlob> blobs;
  for (auto& lv : sp.levels) {
    lv.nbatches = 0;
    all.push_back(&lv.stack);
    all.push_back(&lv.wproj);
    all.push_back(&lv.strips);
    for (auto& g : lv.close1) all.push_back(&g);
    for (auto& g : lv.close2) all.push_back(&g);
    for (auto& g : lv.coup1) all.push_back(&g);
    for (auto& g : lv.coup2) all.push_back(&g);
    blobs.push_back({lv.qr.items.data(), lv.qr.items.size() * sizeof(QrItem),
                     reinterpret_cast<const void**>(&lv.qr.d_items)});
    lv.nbatches = int(all.size());  // batches of this level and the ones below
  }
  // stack and wproj (the basis QR's input) run in FP64, the transforms in the
  // precision of S
  for (GemmBatch* g : all) {
    g->set_generator(dim, H->kern, H->scale, H->diag, H->kparam);
    g->prec = sp.precision == H2_MIXED ? 1 : 0;
  }
  for (auto& lv : sp.levels) lv.stack.prec = lv.wproj.prec = 0;
  tt.lap("work-lists");
  HIPCHECK(hipStreamSynchronize(current_stream()));
  if (!upload) return spp.release();  // a batched sweep merges and uploads the lists
  // the leaf level's lists now; the others during the leaf level's kernels
  // (run_levels), so that their copy overlaps device work
  {
    const size_t n0 = size_t(sp.levels[0].nbatches);
    std::vector<GemmBatch*> first(all.begin(), all.begin() + n0);
    std::vector<RawBlob> firstb(blobs.begin(), blobs.begin() + 1);
    upload_batches(first, sp.dDesc, firstb);
    std::vector<QrItem>().swap(sp.levels[0].qr.items);
    sp.upload_rest = all.size() > n0;
  }
  tt.lap("upload");
  return spp.release();
}

// Uploads the work lists of levels 1..L on a copy stream; `st` waits for the
// copy, after the leaf level's kernels already queued on it.
static void upload_rest(h2_sparse& sp, hipStream_t st) {
  std::vector<GemmBatch*> all;
  std::vector<RawBlob> blobs;
  for (size_t k = 1; k < sp.levels.size(); ++k) {
    SweepLevel& lv = sp.levels[k];
    all.push_back(&lv.stack);
    all.push_back(&lv.wproj);
    all.push_back(&lv.strips);
    for (auto& g : lv.close1) all.push_back(&g);
    for (auto& g : lv.close2) all.push_back(&g);
    for (auto& g : lv.coup1) all.push_back(&g);
    for (auto& g : lv.coup2) all.push_back(&g);
    blobs.push_back({lv.qr.items.data(), lv.qr.items.size() * sizeof(QrItem),
                     reinterpret_cast<const void**>(&lv.qr.d_items)});
  }
  hipStream_t copy = nullptr;
  HIPCHECK(hipStreamCreateWithFlags(&copy, hipStreamNonBlocking));
  try {
    upload_batches(all, sp.dDesc2, blobs, copy, st);
  } catch (...) {
    (void)hipStreamSynchronize(copy);
    (void)hipStreamDestroy(copy);
    throw;
  }
  (void)hipStreamDestroy(copy);  // upload_batches made st wait for the copy
  for (size_t k = 1; k < sp.levels.size(); ++k) std::vector<QrItem>().swap(sp.levels[k].qr.items);
  sp.upload_rest = false;
}

template <class T>
static void run_levels(h2_sparse& sp, hipStream_t st, double* phase_ms) {
  h2_matrix& H = *sp.H;
  const int L = H.tree.depth;
  const bool mixed = sp.precision == H2_MIXED;
  std::vector<hipEvent_t> ev;
  auto mark = [&]() {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    HIPCHECK(hipEventRecord(e, st));
    ev.push_back(e);
  };
  mark();
  for (int k = 0; k <= L; ++k) {
    SweepLevel& lv = sp.levels[k];
    launch_qr(lv.qr.d_items, lv.qr.count, st);
    lv.stack.launch<double>(st);
    lv.wproj.launch<double>(st);
    if (mixed) {
      launch_cast_d2f(sp.dQ.as<double>() + lv.qr.q_begin, sp.dQt.as<float>() + lv.qr.q_begin,
                      lv.qr.q_end - lv.qr.q_begin, st);
      const double* wsrc = H.identity_proj ? sp.dRhat.as<double>() : sp.dW.as<double>();
      launch_cast_d2f(wsrc + lv.qr.w_begin, sp.dWt.as<float>() + lv.qr.w_begin, lv.qr.w_end - lv.qr.w_begin, st);
    }
    mark();  // QR phase end
    if (lv.gnext_entries > 0) {
      if (mixed) launch_fill_f(sp.dG[lv.gnext_side].as<float>(), lv.gnext_entries, 0.0f, st);
      else launch_fill(sp.dG[lv.gnext_side].as<double>(), lv.gnext_entries, 0.0, st);
    }
    lv.strips.launch<T>(st);
    mark();  // strips end
    for (size_t c = 0; c < lv.close1.size(); ++c) {
      lv.close1[c].launch<T>(st);
      lv.close2[c].launch<T>(st);
    }
    mark();  // close end
    for (size_t c = 0; c < lv.coup1.size(); ++c) {
      lv.coup1[c].launch<T>(st);
      lv.coup2[c].launch<T>(st);
    }
    mark();  // couplings end
    if (k == 0 && sp.upload_rest) upload_rest(sp, st);
  }
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipEventSynchronize(ev.back()));
  double acc[4] = {0, 0, 0, 0};  // QR, strips, close, couplings
  for (int k = 0; k <= L; ++k)
    for (int ph = 0; ph < 4; ++ph) {
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, ev[4 * k + ph], ev[4 * k + ph + 1]));
      acc[ph] += ms;
    }
  float tot = 0;
  HIPCHECK(hipEventElapsedTime(&tot, ev.front(), ev.back()));
  for (auto e : ev) (void)hipEventDestroy(e);
  if (phase_ms) {
    phase_ms[0] = acc[0];
    phase_ms[1] = acc[2];
    phase_ms[2] = acc[3];
    phase_ms[3] = acc[1];
    phase_ms[6] = tot;
  }
}

void run_sparsify(h2_sparse& sp, hipStream_t st, double* phase_ms) {
  if (sp.precision == H2_MIXED) run_levels<float>(sp, st, phase_ms);
  else run_levels<double>(sp, st, phase_ms);
}

h2_sparse* plan_sparsify(h2_matrix* H, int precision, bool upload) { return plan(H, precision, upload); }
h2_sparse* plan_symbolic(h2_matrix* H) { return plan(H, H2_FP64, false, true); }

// Several sparsifications swept together (independent H^2 matrices of uneven
// size): level k of every instance goes into the same launches.  Work items
// carry absolute addresses and their own kernel constants, so the instances'
// lists are concatenated per step and chunk and every instance keeps its own
// arenas; only the per-instance casts and arena clears stay separate.
struct MergedLevel {
  std::vector<QrItem> qr;
  const QrItem* d_qr = nullptr;
  int nqr = 0;
  GemmBatch stack, wproj, strips;
  std::vector<GemmBatch> close1, close2, coup1, coup2;
};

template <class T>
static void run_merged(std::vector<h2_sparse*>& sps, std::vector<MergedLevel>& M, hipStream_t st,
                       double* phase_ms) {
  const bool mixed = sps.front()->precision == H2_MIXED;
  std::vector<hipEvent_t> ev;
  auto mark = [&]() {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    HIPCHECK(hipEventRecord(e, st));
    ev.push_back(e);
  };
  mark();
  const int nlev = int(M.size());
  for (int k = 0; k < nlev; ++k) {
    MergedLevel& m = M[k];
    launch_qr(m.d_qr, m.nqr, st);
    m.stack.launch<double>(st);
    m.wproj.launch<double>(st);
    for (h2_sparse* sp : sps) {
      if (k > sp->H->tree.depth || !mixed) continue;
      const SweepLevel& lv = sp->levels[k];
      launch_cast_d2f(sp->dQ.as<double>() + lv.qr.q_begin, sp->dQt.as<float>() + lv.qr.q_begin,
                      lv.qr.q_end - lv.qr.q_begin, st);
      const double* wsrc = sp->H->identity_proj ? sp->dRhat.as<double>() : sp->dW.as<double>();
      launch_cast_d2f(wsrc + lv.qr.w_begin, sp->dWt.as<float>() + lv.qr.w_begin, lv.qr.w_end - lv.qr.w_begin, st);
    }
    mark();
    for (h2_sparse* sp : sps) {
      if (k > sp->H->tree.depth) continue;
      const SweepLevel& lv = sp->levels[k];
      if (lv.gnext_entries <= 0) continue;
      if (mixed) launch_fill_f(sp->dG[lv.gnext_side].as<float>(), lv.gnext_entries, 0.0f, st);
      else launch_fill(sp->dG[lv.gnext_side].as<double>(), lv.gnext_entries, 0.0, st);
    }
    m.strips.launch<T>(st);
    mark();
    for (size_t c = 0; c < m.close1.size(); ++c) {
      m.close1[c].launch<T>(st);
      m.close2[c].launch<T>(st);
    }
    mark();
    for (size_t c = 0; c < m.coup1.size(); ++c) {
      m.coup1[c].launch<T>(st);
      m.coup2[c].launch<T>(st);
    }
    mark();
  }
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipEventSynchronize(ev.back()));
  double acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < nlev; ++k)
    for (int ph = 0; ph < 4; ++ph) {
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, ev[4 * k + ph], ev[4 * k + ph + 1]));
      acc[ph] += ms;
    }
  float tot = 0;
  HIPCHECK(hipEventElapsedTime(&tot, ev.front(), ev.back()));
  for (auto e : ev) (void)hipEventDestroy(e);
  if (phase_ms) {
    phase_ms[0] = acc[0];
    phase_ms[1] = acc[2];
    phase_ms[2] = acc[3];
    phase_ms[3] = acc[1];
    phase_ms[6] = tot;
  }
}

void run_sparsify_batch(std::vector<h2_sparse*>& sps, hipStream_t st, double* phase_ms) {
  TraceTimer tt("sparsify-batch");
  int nlev = 0;
  for (h2_sparse* sp : sps) nlev = std::max(nlev, sp->H->tree.depth + 1);
  std::vector<MergedLevel> M(nlev);
  // levels merge independently (in parallel); inside a level the instances
  // follow in order, each batch sized once before the copies
  int err_code = 0;
  std::string err_msg;
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < nlev; ++k) {
    try {
      MergedLevel& m = M[k];
      size_t nq = 0, nchunk[4] = {0, 0, 0, 0};
      for (h2_sparse* sp : sps) {
        if (k > sp->H->tree.depth) continue;
        const SweepLevel& lv = sp->levels[k];
        nq += lv.qr.items.size();
        nchunk[0] = std::max(nchunk[0], lv.close1.size());
        nchunk[1] = std::max(nchunk[1], lv.close2.size());
        nchunk[2] = std::max(nchunk[2], lv.coup1.size());
        nchunk[3] = std::max(nchunk[3], lv.coup2.size());
      }
      m.qr.reserve(nq);
      m.close1.resize(nchunk[0]);
      m.close2.resize(nchunk[1]);
      m.coup1.resize(nchunk[2]);
      m.coup2.resize(nchunk[3]);
      auto reserve = [&](GemmBatch& dst, auto pick) {
        size_t ni = 0, ns = 0;
        for (h2_sparse* sp : sps) {
          if (k > sp->H->tree.depth) continue;
          const GemmBatch* b = pick(sp->levels[k]);
          if (b) ni += b->items.size(), ns += b->segs.size();
        }
        dst.items.reserve(ni);
        dst.segs.reserve(ns);
      };
      reserve(m.stack, [](SweepLevel& lv) -> const GemmBatch* { return &lv.stack; });
      reserve(m.wproj, [](SweepLevel& lv) -> const GemmBatch* { return &lv.wproj; });
      reserve(m.strips, [](SweepLevel& lv) -> const GemmBatch* { return &lv.strips; });
      for (size_t c = 0; c < nchunk[0]; ++c)
        reserve(m.close1[c], [c](SweepLevel& lv) -> const GemmBatch* { return c < lv.close1.size() ? &lv.close1[c] : nullptr; });
      for (size_t c = 0; c < nchunk[1]; ++c)
        reserve(m.close2[c], [c](SweepLevel& lv) -> const GemmBatch* { return c < lv.close2.size() ? &lv.close2[c] : nullptr; });
      for (size_t c = 0; c < nchunk[2]; ++c)
        reserve(m.coup1[c], [c](SweepLevel& lv) -> const GemmBatch* { return c < lv.coup1.size() ? &lv.coup1[c] : nullptr; });
      for (size_t c = 0; c < nchunk[3]; ++c)
        reserve(m.coup2[c], [c](SweepLevel& lv) -> const GemmBatch* { return c < lv.coup2.size() ? &lv.coup2[c] : nullptr; });
      for (h2_sparse* sp : sps) {
        if (k > sp->H->tree.depth) continue;
        SweepLevel& lv = sp->levels[k];
        m.qr.insert(m.qr.end(), lv.qr.items.begin(), lv.qr.items.end());
        std::vector<QrItem>().swap(lv.qr.items);
        m.stack.append(lv.stack);
        m.wproj.append(lv.wproj);
        m.strips.append(lv.strips);
        for (size_t c = 0; c < lv.close1.size(); ++c) m.close1[c].append(lv.close1[c]);
        for (size_t c = 0; c < lv.close2.size(); ++c) m.close2[c].append(lv.close2[c]);
        for (size_t c = 0; c < lv.coup1.size(); ++c) m.coup1[c].append(lv.coup1[c]);
        for (size_t c = 0; c < lv.coup2.size(); ++c) m.coup2[c].append(lv.coup2[c]);
      }
      m.nqr = int(m.qr.size());
    } catch (const Error& e) {
#pragma omp critical(h2_merge_error)
      if (!err_code) err_code = e.code, err_msg = e.msg;
    }
  }
  if (err_code) fail(err_code, err_msg);
  tt.lap("merge");
  std::vector<GemmBatch*> all;
  std::vector<RawBlob> blobs;
  for (MergedLevel& m : M) {
    all.push_back(&m.stack);
    all.push_back(&m.wproj);
    all.push_back(&m.strips);
    for (auto& g : m.close1) all.push_back(&g);
    for (auto& g : m.close2) all.push_back(&g);
    for (auto& g : m.coup1) all.push_back(&g);
    for (auto& g : m.coup2) all.push_back(&g);
    blobs.push_back({m.qr.data(), m.qr.size() * sizeof(QrItem), reinterpret_cast<const void**>(&m.d_qr)});
  }
  for (GemmBatch* g : all) g->prec = sps.front()->precision == H2_MIXED ? 1 : 0;
  for (MergedLevel& m : M) m.stack.prec = m.wproj.prec = 0;
  DeviceBuffer desc;
  upload_batches(all, desc, blobs);
  tt.lap("upload");
  if (sps.front()->precision == H2_MIXED) run_merged<float>(sps, M, st, phase_ms);
  else run_merged<double>(sps, M, st, phase_ms);
  tt.lap("run");
}

}  // namespace h2
