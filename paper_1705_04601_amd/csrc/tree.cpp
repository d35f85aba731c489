// Cluster tree and block cluster tree (Section 4.1, Definitions 4.1-4.4).
//
// kd-tree: all leaves at depth L = smallest L with ceil(n / 2^L) <= leaf; a
// cluster is split along the longest axis of its tight box (lowest axis on
// ties), its points ordered by (coordinate, original index), the first
// floor(n/2) going to the left son.  The order is a total order, so the result
// does not depend on the sorting algorithm.
//
// Admissibility: t != s, d^2 > 0 and d^2 >= eta^2 max(diam_t^2, diam_s^2) on
// tight boxes, each sum accumulated in axis order; eta = 0 is weak
// admissibility (t != s).  This file is compiled with -ffp-contract=off so that
// the comparisons are reproducible operation by operation.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "h2_internal.h"

namespace h2 {

int Tree::level(i64 c) const {
  int d = 0;
  for (i64 v = c + 1; v > 1; v >>= 1) ++d;
  return depth - d;
}

Tree build_tree(const double* pts, i64 n, int dim, int leaf) {
  Tree tr;
  tr.n = n;
  tr.dim = dim;
  int depth = 0;
  while (((n + (i64(1) << depth) - 1) >> depth) > leaf) ++depth;
  tr.depth = depth;
  const i64 ncl = tr.ncl();
  tr.start.assign(ncl, 0);
  tr.size.assign(ncl, 0);
  tr.lo.assign(ncl * dim, 0.0);
  tr.hi.assign(ncl * dim, 0.0);
  tr.perm.resize(n);
  std::iota(tr.perm.begin(), tr.perm.end(), i64(0));
  tr.size[0] = n;
  for (i64 c = 0; c < ncl; ++c) {
    const i64 s0 = tr.start[c], sz = tr.size[c];
    i64* idx = tr.perm.data() + s0;
    for (int a = 0; a < dim; ++a) {
      double lo = pts[idx[0] * dim + a], hi = lo;
      for (i64 i = 1; i < sz; ++i) {
        const double v = pts[idx[i] * dim + a];
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
      tr.lo[c * dim + a] = lo;
      tr.hi[c * dim + a] = hi;
    }
    if (2 * c + 1 >= ncl) continue;
    int axis = 0;
    double best = tr.hi[c * dim] - tr.lo[c * dim];
    for (int a = 1; a < dim; ++a) {
      const double e = tr.hi[c * dim + a] - tr.lo[c * dim + a];
      if (e > best) { best = e; axis = a; }
    }
    std::sort(idx, idx + sz, [&](i64 u, i64 v) {
      const double pu = pts[u * dim + axis], pv = pts[v * dim + axis];
      return pu < pv || (pu == pv && u < v);
    });
    const i64 nl = sz / 2;
    tr.start[2 * c + 1] = s0;
    tr.size[2 * c + 1] = nl;
    tr.start[2 * c + 2] = s0 + nl;
    tr.size[2 * c + 2] = sz - nl;
  }
  return tr;
}

static bool admissible(const Tree& tr, i64 t, i64 s, double eta) {
  if (t == s) return false;
  if (eta == 0.0) return true;
  const int dim = tr.dim;
  double d2 = 0.0, dt2 = 0.0, ds2 = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double g = std::max(0.0, std::max(tr.lo[s * dim + a] - tr.hi[t * dim + a],
                                            tr.lo[t * dim + a] - tr.hi[s * dim + a]));
    d2 = d2 + g * g;
    const double et = tr.hi[t * dim + a] - tr.lo[t * dim + a];
    const double es = tr.hi[s * dim + a] - tr.lo[s * dim + a];
    dt2 = dt2 + et * et;
    ds2 = ds2 + es * es;
  }
  const double bound = std::max(dt2, ds2) * (eta * eta);
  return d2 > 0.0 && d2 >= bound;
}

BlockTree build_block_tree(const Tree& tr, double eta) {
  BlockTree bt;
  const int L = tr.depth;
  bt.near.resize(L + 1);
  bt.far.resize(L + 1);
  std::vector<Pair> cur{{0, 0}};
  auto by_ts = [](const Pair& a, const Pair& b) { return a.t < b.t || (a.t == b.t && a.s < b.s); };
  for (int k = L; k >= 0; --k) {
    auto& nr = bt.near[k];
    auto& fr = bt.far[k];
    for (const Pair& p : cur) (admissible(tr, p.t, p.s, eta) ? fr : nr).push_back(p);
    std::sort(nr.begin(), nr.end(), by_ts);
    std::sort(fr.begin(), fr.end(), by_ts);
    if (k == 0) break;
    std::vector<Pair> next;
    next.reserve(nr.size() * 4);
    for (const Pair& p : nr)
      for (int a = 1; a <= 2; ++a)
        for (int b = 1; b <= 2; ++b) next.push_back({2 * p.t + a, 2 * p.s + b});
    cur.swap(next);
  }
  return bt;
}

std::vector<char> farfield_flags(const Tree& tr, const BlockTree& bt) {
  std::vector<char> ff(tr.ncl(), 0);
  for (const auto& lev : bt.far)
    for (const Pair& p : lev) ff[p.t] = 1;
  for (i64 c = 1; c < tr.ncl(); ++c)
    if (ff[(c - 1) / 2]) ff[c] = 1;
  return ff;
}

}  // namespace h2
