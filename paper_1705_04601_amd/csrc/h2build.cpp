// Construction of the H^2 matrix of c/|x - y|, c exp(-|x - y|^2) or the kernel of Example 5.4
// (c r / d below d, c d / r from d on; Section 5.5) (the input of the method,
// Definition 4.9 (the H^2 matrix); the paper takes it as given and cites H^2 compression for
// orthogonal nested bases in Section 4.2).
//
// * Tensor Chebyshev nodes of the first kind (p per axis) on each cluster's
//   tight box (a zero-width axis widened by 1e-12 max(1, |lo|)); leaf basis =
//   Lagrange polynomials at the points, transfer = father's Lagrange
//   polynomials at the son's nodes, coupling = kernel at the nodes.
// * Recompression: orthogonalise the nested basis (QR per cluster, bottom-up),
//   accumulate each cluster's farfield weight top-down (R factor of the stacked
//   couplings and the father's weight), truncate bottom-up by the SVD of the
//   weighted basis (one-sided Jacobi), keeping sigma_i > tol * sigma_1, at most
//   rank_cap, at least one.  Couplings are then P_t K_ts P_s^T.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "h2_internal.h"

namespace h2 {
namespace {

// Column-major dense matrix on the host.
struct Mat {
  int m = 0, n = 0;
  std::vector<double> a;
  Mat() = default;
  Mat(int m_, int n_) : m(m_), n(n_), a(size_t(m_) * n_, 0.0) {}
  double& operator()(int i, int j) { return a[size_t(j) * m + i]; }
  double operator()(int i, int j) const { return a[size_t(j) * m + i]; }
};

// C = op(A) op(B); op = transpose when the flag is set.
Mat mul(const Mat& A, bool ta, const Mat& B, bool tb) {
  const int m = ta ? A.n : A.m, k = ta ? A.m : A.n;
  const int n = tb ? B.m : B.n;
  Mat C(m, n);
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < k; ++l) {
      const double b = tb ? B(j, l) : B(l, j);
      if (b == 0.0) continue;
      double* c = &C.a[size_t(j) * m];
      if (!ta) {
        const double* acol = &A.a[size_t(l) * A.m];
        for (int i = 0; i < m; ++i) c[i] += acol[i] * b;
      } else {
        for (int i = 0; i < m; ++i) c[i] += A(l, i) * b;
      }
    }
  return C;
}

Mat vstack(const Mat& a, const Mat& b) {
  Mat c(a.m + b.m, a.n);
  for (int j = 0; j < a.n; ++j) {
    for (int i = 0; i < a.m; ++i) c(i, j) = a(i, j);
    for (int i = 0; i < b.m; ++i) c(a.m + i, j) = b(i, j);
  }
  return c;
}

// Householder QR: A (m x n) = Q R with Q (m x q) orthonormal columns, R (q x n),
// q = min(m, n).  Q is formed only when wanted.
void qr(const Mat& A, Mat* Q, Mat* R) {
  Mat w = A;
  const int m = w.m, n = w.n, q = std::min(m, n);
  std::vector<double> tau(q, 0.0);
  for (int j = 0; j < q; ++j) {
    double s = 0.0;
    for (int i = j + 1; i < m; ++i) s += w(i, j) * w(i, j);
    const double alpha = w(j, j);
    if (s == 0.0) { tau[j] = 0.0; continue; }
    const double nrm = std::sqrt(alpha * alpha + s);
    const double beta = alpha >= 0.0 ? -nrm : nrm;
    tau[j] = (beta - alpha) / beta;
    const double sc = 1.0 / (alpha - beta);
    for (int i = j + 1; i < m; ++i) w(i, j) *= sc;
    w(j, j) = beta;
    for (int c = j + 1; c < n; ++c) {
      double d = w(j, c);
      for (int i = j + 1; i < m; ++i) d += w(i, j) * w(i, c);
      d *= tau[j];
      w(j, c) -= d;
      for (int i = j + 1; i < m; ++i) w(i, c) -= d * w(i, j);
    }
  }
  if (R) {
    *R = Mat(q, n);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i <= std::min(j, q - 1); ++i) (*R)(i, j) = w(i, j);
  }
  if (Q) {
    *Q = Mat(m, q);
    for (int j = 0; j < q; ++j) (*Q)(j, j) = 1.0;
    for (int j = q - 1; j >= 0; --j) {
      if (tau[j] == 0.0) continue;
      for (int c = j; c < q; ++c) {
        double d = (*Q)(j, c);
        for (int i = j + 1; i < m; ++i) d += w(i, j) * (*Q)(i, c);
        d *= tau[j];
        (*Q)(j, c) -= d;
        for (int i = j + 1; i < m; ++i) (*Q)(i, c) -= d * w(i, j);
      }
    }
  }
}

// Left singular vectors (columns sorted by decreasing sigma) of Y (m x n) by
// one-sided Jacobi rotations on the columns (Hestenes).
void svd_left(const Mat& Y, Mat* U, std::vector<double>* sig) {
  Mat a = Y;
  const int m = a.m, n = a.n;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q2 = p + 1; q2 < n; ++q2) {
        double app = 0, aqq = 0, apq = 0;
        for (int i = 0; i < m; ++i) {
          const double x = a(i, p), y = a(i, q2);
          app += x * x;
          aqq += y * y;
          apq += x * y;
        }
        if (apq == 0.0 || std::fabs(apq) <= 1e-15 * std::sqrt(app * aqq)) continue;
        rotated = true;
        const double zeta = (aqq - app) / (2.0 * apq);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          const double x = a(i, p), y = a(i, q2);
          a(i, p) = c * x - s * y;
          a(i, q2) = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
  std::vector<double> nrm(n);
  std::vector<int> ord(n);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += a(i, j) * a(i, j);
    nrm[j] = std::sqrt(s);
    ord[j] = j;
  }
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
  const int r = std::min(m, n);
  *U = Mat(m, r);
  sig->assign(r, 0.0);
  for (int k = 0; k < r; ++k) {
    const int j = ord[k];
    (*sig)[k] = nrm[j];
    if (nrm[j] > 0)
      for (int i = 0; i < m; ++i) (*U)(i, k) = a(i, j) / nrm[j];
  }
  // Columns belonging to zero singular values are completed to an orthonormal
  // set by Gram-Schmidt against unit vectors (only their span matters).
  for (int k = 0; k < r; ++k) {
    if ((*sig)[k] > 0) continue;
    for (int e = 0; e < m; ++e) {
      std::vector<double> v(m, 0.0);
      v[e] = 1.0;
      for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l < r; ++l) {
          if (l == k || ((*sig)[l] == 0 && l > k)) continue;
          double d = 0;
          for (int i = 0; i < m; ++i) d += (*U)(i, l) * v[i];
          for (int i = 0; i < m; ++i) v[i] -= d * (*U)(i, l);
        }
      double s = 0;
      for (int i = 0; i < m; ++i) s += v[i] * v[i];
      if (s > 0.5) {
        s = std::sqrt(s);
        for (int i = 0; i < m; ++i) (*U)(i, k) = v[i] / s;
        break;
      }
    }
  }
}

void cheb_axis(double lo, double hi, int p, double* out) {
  for (int i = 0; i < p; ++i)
    out[i] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * std::cos((2 * i + 1) * M_PI / (2 * p));
}

// Box of cluster c, zero-width axes widened.
void padded_box(const Tree& tr, i64 c, double* lo, double* hi) {
  for (int a = 0; a < tr.dim; ++a) {
    lo[a] = tr.lo[c * tr.dim + a];
    hi[a] = tr.hi[c * tr.dim + a];
    if (hi[a] == lo[a]) {
      const double d = 1e-12 * std::max(1.0, std::fabs(lo[a]));
      lo[a] -= d;
      hi[a] += d;
    }
  }
}

// Tensor Lagrange basis of box (lo, hi) evaluated at m points (row-major m x dim):
// returns m x p^dim, column index nu = i0 + p i1 + p^2 i2.
Mat lagrange(const double* lo, const double* hi, int dim, int p, const double* pts, int m) {
  int P = 1;
  for (int a = 0; a < dim; ++a) P *= p;
  Mat out(m, P);
  double nodes[3][8];
  for (int a = 0; a < dim; ++a) cheb_axis(lo[a], hi[a], p, nodes[a]);
  std::vector<double> l1(size_t(dim) * p);
  for (int r = 0; r < m; ++r) {
    for (int a = 0; a < dim; ++a) {
      const double x = pts[r * dim + a];
      for (int i = 0; i < p; ++i) {
        double v = 1.0;
        for (int j = 0; j < p; ++j)
          if (j != i) v *= (x - nodes[a][j]) / (nodes[a][i] - nodes[a][j]);
        l1[a * p + i] = v;
      }
    }
    for (int nu = 0; nu < P; ++nu) {
      int rem = nu;
      double v = 1.0;
      for (int a = 0; a < dim; ++a) {
        v *= l1[a * p + rem % p];
        rem /= p;
      }
      out(r, nu) = v;
    }
  }
  return out;
}

Mat kernel_at_nodes(const double* xr, const double* xc, int P, int dim, int kern, double scale, double param) {
  Mat k(P, P);
  for (int j = 0; j < P; ++j)
    for (int i = 0; i < P; ++i) {
      double d2 = 0;
      for (int a = 0; a < dim; ++a) {
        const double d = xr[i * dim + a] - xc[j * dim + a];
        d2 += d * d;
      }
      if (kern == H2_KERNEL_EXP) {
        k(i, j) = scale * std::exp(-d2);
      } else if (kern == H2_KERNEL_IFMM) {
        const double r = std::sqrt(d2);  // Example 5.4: r / d below d, d / r from d on
        k(i, j) = r < param ? scale * (r / param) : scale * (param / r);
      } else {
        k(i, j) = scale / std::sqrt(d2);
      }
    }
  return k;
}

}  // namespace

void fill_structure(h2_matrix& H, const double* pts, i64 n, int dim, const h2_kernel& kern,
                    const h2_build_opts& o) {
  H.tree = build_tree(pts, n, dim, o.leaf);
  H.bt = build_block_tree(H.tree, o.eta);
  H.ff = farfield_flags(H.tree, H.bt);
  H.x_tree.resize(size_t(n) * dim);
  for (i64 i = 0; i < n; ++i)
    for (int a = 0; a < dim; ++a) H.x_tree[i * dim + a] = pts[H.tree.perm[i] * dim + a];
  H.scale = kern.scale;
  H.kern = kern.kind;
  H.kparam = kern.kind == H2_KERNEL_IFMM ? kern.param : 0.0;
  H.diag = kern.diag;
  H.cheb = o.cheb;
  H.P = 1;
  for (int a = 0; a < dim; ++a) H.P *= o.cheb;
  const i64 ncl = H.tree.ncl();
  H.nodes.assign(size_t(ncl) * H.P * dim, 0.0);
#pragma omp parallel for schedule(dynamic, 64)
  for (i64 c = 0; c < ncl; ++c) {
    if (!H.ff[c]) continue;
    double lo[3], hi[3], ax[3][8];
    padded_box(H.tree, c, lo, hi);
    for (int a = 0; a < dim; ++a) cheb_axis(lo[a], hi[a], o.cheb, ax[a]);
    for (int nu = 0; nu < H.P; ++nu) {
      int rem = nu;
      for (int a = 0; a < dim; ++a) {
        H.nodes[(size_t(c) * H.P + nu) * dim + a] = ax[a][rem % o.cheb];
        rem /= o.cheb;
      }
    }
  }
}

void build_chebyshev(h2_matrix& H, double tol, int rank_cap) {
  const Tree& tr = H.tree;
  const int dim = tr.dim, P = H.P, p = H.cheb;
  const i64 ncl = tr.ncl();
  const double* nodes = H.nodes.data();
  auto node_ptr = [&](i64 c) { return nodes + size_t(c) * P * dim; };

  // Chebyshev leaf bases V_t and transfers E_c.
  std::vector<Mat> V(ncl), E(ncl);
#pragma omp parallel for schedule(dynamic, 16)
  for (i64 c = 0; c < ncl; ++c) {
    if (!H.ff[c]) continue;
    if (tr.is_leaf(c)) {
      double lo[3], hi[3];
      padded_box(tr, c, lo, hi);
      V[c] = lagrange(lo, hi, dim, p, H.x_tree.data() + tr.start[c] * dim, int(tr.size[c]));
    }
    if (c > 0 && H.ff[(c - 1) / 2]) {
      double lo[3], hi[3];
      padded_box(tr, (c - 1) / 2, lo, hi);
      E[c] = lagrange(lo, hi, dim, p, node_ptr(c), P);
    }
  }

  std::vector<Mat> leafB(ncl), T(ncl), Pm(ncl);
  H.rank.assign(ncl, 0);
  if (tol <= 0.0) {
    H.identity_proj = true;
    for (i64 c = 0; c < ncl; ++c) {
      if (!H.ff[c]) continue;
      H.rank[c] = P;
      if (tr.is_leaf(c)) leafB[c] = std::move(V[c]);
      if (c > 0 && H.ff[(c - 1) / 2]) T[c] = std::move(E[c]);
      Pm[c] = Mat(P, P);
      for (int i = 0; i < P; ++i) Pm[c](i, i) = 1.0;
    }
  } else {
    H.identity_proj = false;
    const int L = tr.depth;
    // R1: orthogonalise bottom-up.  V_t = Phi_t Z_t; Phi_father = diag(Phi_c) Psi.
    std::vector<Mat> Z(ncl), Psi(ncl), PhiLeaf(ncl);
    for (int k = 0; k <= L; ++k) {
      const i64 f = tr.first_at_level(k), cnt = tr.count_at_level(k);
#pragma omp parallel for schedule(dynamic, 8)
      for (i64 c = f; c < f + cnt; ++c) {
        if (!H.ff[c]) continue;
        Mat M = (k == 0) ? V[c]
                         : vstack(mul(Z[2 * c + 1], false, E[2 * c + 1], false),
                                  mul(Z[2 * c + 2], false, E[2 * c + 2], false));
        Mat Q, R;
        qr(M, &Q, &R);
        Z[c] = std::move(R);
        if (k == 0) {
          PhiLeaf[c] = std::move(Q);
        } else {
          const int k1 = Z[2 * c + 1].m;
          Mat q1(k1, Q.n), q2(Q.m - k1, Q.n);
          for (int j = 0; j < Q.n; ++j) {
            for (int i = 0; i < k1; ++i) q1(i, j) = Q(i, j);
            for (int i = k1; i < Q.m; ++i) q2(i - k1, j) = Q(i, j);
          }
          Psi[2 * c + 1] = std::move(q1);
          Psi[2 * c + 2] = std::move(q2);
        }
      }
    }
    // R2: farfield weights top-down.
    std::vector<std::vector<int32_t>> farOf(ncl);
    for (const auto& lev : H.bt.far)
      for (const Pair& pr : lev) farOf[pr.t].push_back(pr.s);
    std::vector<Mat> W(ncl);
    for (int k = L; k >= 0; --k) {
      const i64 f = tr.first_at_level(k), cnt = tr.count_at_level(k);
#pragma omp parallel for schedule(dynamic, 4)
      for (i64 c = f; c < f + cnt; ++c) {
        if (!H.ff[c]) continue;
        const int q = Z[c].m;
        const bool withFather = c > 0 && H.ff[(c - 1) / 2];
        int cols = 0;
        for (int32_t s : farOf[c]) cols += Z[s].m;
        Mat fatherPart;
        if (withFather) {
          fatherPart = mul(Psi[c], false, W[(c - 1) / 2], false);
          cols += fatherPart.n;
        }
        Mat Ft(cols, q);  // F_t^T, stacked
        int off = 0;
        for (int32_t s : farOf[c]) {
          Mat K = kernel_at_nodes(node_ptr(c), node_ptr(s), P, dim, H.kern, H.scale, H.kparam);
          Mat D = mul(mul(Z[c], false, K, false), false, Z[s], true);  // q x q_s
          for (int j = 0; j < q; ++j)
            for (int i = 0; i < D.n; ++i) Ft(off + i, j) = D(j, i);
          off += D.n;
        }
        if (withFather)
          for (int j = 0; j < q; ++j)
            for (int i = 0; i < fatherPart.n; ++i) Ft(off + i, j) = fatherPart(j, i);
        Mat R;
        qr(Ft, nullptr, &R);
        // W = R^T (q x min(cols, q))
        Mat Wc(q, R.m);
        for (int i = 0; i < R.m; ++i)
          for (int j = 0; j < q; ++j) Wc(j, i) = R(i, j);
        W[c] = std::move(Wc);
      }
    }
    // R3: truncation bottom-up.
    std::vector<Mat> Pi(ncl);
    for (int k = 0; k <= L; ++k) {
      const i64 f = tr.first_at_level(k), cnt = tr.count_at_level(k);
#pragma omp parallel for schedule(dynamic, 8)
      for (i64 c = f; c < f + cnt; ++c) {
        if (!H.ff[c]) continue;
        Mat Yhat;
        if (k == 0) {
          Yhat = Mat(Z[c].m, Z[c].m);
          for (int i = 0; i < Z[c].m; ++i) Yhat(i, i) = 1.0;
        } else {
          Yhat = vstack(mul(Pi[2 * c + 1], false, Psi[2 * c + 1], false),
                        mul(Pi[2 * c + 2], false, Psi[2 * c + 2], false));
        }
        Mat U;
        std::vector<double> sig;
        svd_left(mul(Yhat, false, W[c], false), &U, &sig);
        int keep = 0;
        if (!sig.empty() && sig[0] > 0)
          for (double sv : sig) keep += sv > tol * sig[0];
        keep = std::max(1, keep);
        if (rank_cap > 0) keep = std::min(keep, rank_cap);
        keep = std::min(keep, U.n);
        Mat Uk(U.m, keep);
        for (int j = 0; j < keep; ++j)
          for (int i = 0; i < U.m; ++i) Uk(i, j) = U(i, j);
        H.rank[c] = keep;
        Pi[c] = mul(Uk, true, Yhat, false);
        if (k == 0) {
          leafB[c] = mul(PhiLeaf[c], false, Uk, false);
        } else {
          // the sons' new ranks are final (computed on the level below)
          const int k1 = H.rank[2 * c + 1];
          Mat t1(k1, keep), t2(Uk.m - k1, keep);
          for (int j = 0; j < keep; ++j) {
            for (int i = 0; i < k1; ++i) t1(i, j) = Uk(i, j);
            for (int i = k1; i < Uk.m; ++i) t2(i - k1, j) = Uk(i, j);
          }
          T[2 * c + 1] = std::move(t1);
          T[2 * c + 2] = std::move(t2);
        }
        Pm[c] = mul(Pi[c], false, Z[c], false);
      }
    }
  }

  // Flatten into the handle's arrays.
  H.proj_off.assign(ncl, -1);
  H.basis_off.assign(ncl, -1);
  H.transfer_off.assign(ncl, -1);
  H.proj.clear();
  H.basis.clear();
  H.transfer.clear();
  for (i64 c = 0; c < ncl; ++c) {
    if (!H.ff[c]) continue;
    H.proj_off[c] = i64(H.proj.size());
    H.proj.insert(H.proj.end(), Pm[c].a.begin(), Pm[c].a.end());
    if (tr.is_leaf(c)) {
      H.basis_off[c] = i64(H.basis.size());
      H.basis.insert(H.basis.end(), leafB[c].a.begin(), leafB[c].a.end());
    }
    if (c > 0 && H.ff[(c - 1) / 2]) {
      H.transfer_off[c] = i64(H.transfer.size());
      H.transfer.insert(H.transfer.end(), T[c].a.begin(), T[c].a.end());
    }
  }
}

}  // namespace h2
