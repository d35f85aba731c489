"""Oracle: H^2 matrix of the kernel c/|x-y| (or c exp(-|x-y|^2)) by Chebyshev interpolation (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package.

The H^2 format is Definition 4.9 (with Definitions 4.5-4.8): the matrix is
the close part (kernel entries of the nearfield leaf pairs) plus, for every
farfield pair (t, s), R_t D_ts E_s^T with nested cluster bases.  The kernel
is symmetric and one cluster tree serves rows and columns, so E = R.

Construction (the paper takes the H^2 matrix as given, Section 4.1; this is
the reading used here):

* tensor Chebyshev nodes of the first kind, ``p`` per axis, on each
  cluster's tight box; leaf basis = Lagrange polynomials at the points;
  transfer of a son = father's Lagrange polynomials at the son's nodes
  (nestedness is then exact for polynomials); coupling = kernel at the two
  clusters' nodes;
* optional recompression (the H^2 compression cited in Section 4.2):
  orthogonalise the nested basis, form each cluster's total farfield weight
  top-down, truncate bottom-up by the SVD of the weighted basis, keeping
  singular values above ``tol`` times the largest (at most ``rank_cap``,
  at least one).  Couplings become P_t K_ts P_s^T where P_t maps the
  Chebyshev coordinates of t into its new basis.

Only clusters with a nonempty farfield (their own or an ancestor's) carry a
basis; that set is closed under taking sons.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .tree import (BlockTree, ClusterTree, build_block_tree,
                   build_cluster_tree, farfield_nonempty)


EXP = "exp"
IFMM = "ifmm"   # used as (IFMM, d)


def _named_kernel(kernel, r2: np.ndarray, scale: float) -> np.ndarray:
    """Entries of a named kernel at squared distances r2 (off the diagonal).

    EXP: scale exp(-r^2) (Example 5.2).  (IFMM, d): scale r / d for r < d and
    scale d / r otherwise (Example 5.4, the test matrix of Section 5.5).
    """
    if kernel == EXP:
        return scale * np.exp(-r2)
    name, d = kernel
    assert name == IFMM, kernel
    r = np.sqrt(r2)
    with np.errstate(divide="ignore"):
        return scale * np.where(r < d, r / d, d / r)


def _is_named(kernel) -> bool:
    return isinstance(kernel, str) or (isinstance(kernel, tuple) and kernel[:1] == (IFMM,))


def kernel_block(xr: np.ndarray, xc: np.ndarray, scale: float, kernel=None) -> np.ndarray:
    """K_ij = scale / |xr_i - xc_j| for distinct points (no diagonal rule).

    ``kernel`` = EXP gives scale exp(-|xr_i - xc_j|^2), the smooth part of
    the Gaussian matrix of Example 5.2 (the "exp" core, Section 5.1), and
    (IFMM, d) the matrix of Example 5.4 (Section 5.5); a
    function of two point arrays broadcasting to a matrix replaces the
    inverse distance (the tests use polynomial kernels for which Chebyshev
    interpolation is exact).
    """
    diff = xr[:, None, :] - xc[None, :, :]
    if _is_named(kernel):
        return _named_kernel(kernel, (diff * diff).sum(axis=2), scale)
    if kernel is not None:
        return kernel(xr[:, None, :], xc[None, :, :])
    return scale / np.sqrt((diff * diff).sum(axis=2))


def close_block(x: np.ndarray, ti: np.ndarray, si: np.ndarray, scale: float,
                diag: float, kernel=None) -> np.ndarray:
    """Kernel entries A[ti, si] with A_ii = diag (indices into x).

    With kernel = EXP the entries are scale exp(-|x_i - x_j|^2) off the
    diagonal; Example 5.2's matrix 2 delta_ij + exp(-|r_i - r_j|^2) is
    scale = 1, diag = 3.
    """
    if kernel is not None and not _is_named(kernel):
        return kernel(x[ti][:, None, :], x[si][None, :, :])
    diff = x[ti][:, None, :] - x[si][None, :, :]
    r2 = (diff * diff).sum(axis=2)
    same = ti[:, None] == si[None, :]
    if kernel is not None:
        out = _named_kernel(kernel, r2, scale)
    else:
        with np.errstate(divide="ignore"):
            out = scale / np.sqrt(r2)
    out[same] = diag
    return out


def cheb_nodes_1d(a: float, b: float, p: int) -> np.ndarray:
    i = np.arange(p)
    return 0.5 * (a + b) + 0.5 * (b - a) * np.cos((2 * i + 1) * np.pi / (2 * p))


def lagrange_1d(nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """L[m, i] = ell_i(x_m) for the Lagrange polynomials of ``nodes``."""
    p = nodes.shape[0]
    out = np.ones((x.shape[0], p))
    for i in range(p):
        for j in range(p):
            if j != i:
                out[:, i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return out


def padded_box(lo: np.ndarray, hi: np.ndarray):
    """A zero-width axis is widened by 1e-12 * max(1, |lo|) on both sides."""
    lo = lo.copy()
    hi = hi.copy()
    flat = hi == lo
    delta = 1e-12 * np.maximum(1.0, np.abs(lo))
    lo[flat] -= delta[flat]
    hi[flat] += delta[flat]
    return lo, hi


def tensor_nodes(lo: np.ndarray, hi: np.ndarray, p: int) -> np.ndarray:
    """(p^dim, dim) nodes; node index = i0 + p*i1 + p^2*i2."""
    dim = lo.shape[0]
    axes = [cheb_nodes_1d(lo[a], hi[a], p) for a in range(dim)]
    npts = p ** dim
    out = np.empty((npts, dim))
    for nu in range(npts):
        rem = nu
        for a in range(dim):
            out[nu, a] = axes[a][rem % p]
            rem //= p
    return out


def tensor_lagrange(lo: np.ndarray, hi: np.ndarray, p: int, pts: np.ndarray) -> np.ndarray:
    """(m, p^dim) matrix of the tensor Lagrange basis of the box at pts."""
    dim = lo.shape[0]
    per_axis = [lagrange_1d(cheb_nodes_1d(lo[a], hi[a], p), pts[:, a]) for a in range(dim)]
    npts = p ** dim
    out = np.ones((pts.shape[0], npts))
    for nu in range(npts):
        rem = nu
        for a in range(dim):
            out[:, nu] *= per_axis[a][:, rem % p]
            rem //= p
    return out


@dataclass
class H2Matrix:
    tree: ClusterTree
    bt: BlockTree
    ff: np.ndarray            # cluster has a basis
    x_tree: np.ndarray        # points in tree order (n, dim)
    scale: float
    diag: float
    cheb: int
    nodes: dict               # cluster -> (P, dim) Chebyshev nodes
    rank: np.ndarray          # r_t (0 where ff is False)
    leaf_basis: dict          # leaf -> (|t|, r_t)
    transfer: dict            # son c -> (r_c, r_father)
    proj: dict                # t -> (r_t, P): coupling D_ts = P_t K_ts P_s^T
    kernel: object = None     # EXP, or a replacement of the inverse distance

    def coupling(self, t: int, s: int) -> np.ndarray:
        k = kernel_block(self.nodes[t], self.nodes[s], self.scale, self.kernel)
        return self.proj[t] @ k @ self.proj[s].T

    def cluster_slice(self, c: int) -> slice:
        st = int(self.tree.start[c])
        return slice(st, st + int(self.tree.size[c]))

    def expanded_basis(self, t: int) -> np.ndarray:
        """R_t as an |t| x r_t matrix (nested product of transfers)."""
        if 2 * t + 1 >= self.tree.ncl:
            return self.leaf_basis[t]
        parts = [self.expanded_basis(c) @ self.transfer[c] for c in (2 * t + 1, 2 * t + 2)]
        return np.vstack(parts)

    def dense(self) -> np.ndarray:
        """Dense A_H2 in tree order (small n only): Definition 4.9."""
        n = self.tree.n
        a = np.zeros((n, n))
        idx = np.arange(n)
        for t, s in self.bt.near[0]:
            ts, ss = self.cluster_slice(t), self.cluster_slice(s)
            a[ts, ss] = close_block(self.x_tree, idx[ts], idx[ss], self.scale, self.diag, self.kernel)
        for k in range(self.tree.depth + 1):
            for t, s in self.bt.far[k]:
                ts, ss = self.cluster_slice(t), self.cluster_slice(s)
                a[ts, ss] += self.expanded_basis(t) @ self.coupling(t, s) @ self.expanded_basis(s).T
        return a

    def matvec(self, v_tree: np.ndarray) -> np.ndarray:
        """A_H2 @ v for v in tree order (n, nrhs); close part + nested far part."""
        tr = self.tree
        v = v_tree.reshape(tr.n, -1)
        y = np.zeros_like(v)
        idx = np.arange(tr.n)
        for t, s in self.bt.near[0]:
            ts, ss = self.cluster_slice(t), self.cluster_slice(s)
            y[ts] += close_block(self.x_tree, idx[ts], idx[ss], self.scale, self.diag, self.kernel) @ v[ss]
        # upward pass: vhat_t = R_t^T v_t
        vhat = {}
        for lev in range(tr.depth + 1):
            for c in tr.clusters_at_level(lev):
                if not self.ff[c]:
                    continue
                if lev == 0:
                    vhat[c] = self.leaf_basis[c].T @ v[self.cluster_slice(c)]
                else:
                    vhat[c] = sum(self.transfer[s].T @ vhat[s] for s in (2 * c + 1, 2 * c + 2))
        # couplings
        yhat = {c: np.zeros((self.rank[c], v.shape[1])) for c in vhat}
        for k in range(tr.depth + 1):
            for t, s in self.bt.far[k]:
                yhat[t] += self.coupling(t, s) @ vhat[s]
        # downward pass
        for lev in range(tr.depth, -1, -1):
            for c in tr.clusters_at_level(lev):
                if not self.ff[c]:
                    continue
                if c > 0 and self.ff[(c - 1) // 2]:
                    yhat[c] += self.transfer[c] @ yhat[(c - 1) // 2]
                if lev == 0:
                    y[self.cluster_slice(c)] += self.leaf_basis[c] @ yhat[c]
        return y.reshape(v_tree.shape)


def _householder_r(m: np.ndarray) -> np.ndarray:
    """Square-or-short R factor of m (rows >= 1) via LAPACK QR (library step)."""
    return np.linalg.qr(m, mode="r")


def build_h2(x: np.ndarray, leaf: int, cheb: int, scale: float, diag: float = 1.0,
             tol: float = 0.0, rank_cap: int = 0, eta: float = 1.0,
             kernel=None) -> H2Matrix:
    """Chebyshev H^2 of c/|x-y| on points x (original order), optional recompression."""
    tree = build_cluster_tree(x, leaf)
    bt = build_block_tree(tree, eta)
    ff = farfield_nonempty(tree, bt)
    x_tree = np.asarray(x, dtype=np.float64)[tree.perm]
    ncl = tree.ncl
    big_p = cheb ** tree.dim

    boxes = {c: padded_box(tree.lo[c], tree.hi[c]) for c in range(ncl) if ff[c]}
    nodes = {c: tensor_nodes(*boxes[c], cheb) for c in boxes}
    cheb_leaf = {}
    cheb_transfer = {}
    for c in boxes:
        if 2 * c + 1 >= ncl:
            st = int(tree.start[c])
            cheb_leaf[c] = tensor_lagrange(*boxes[c], cheb, x_tree[st:st + tree.size[c]])
        if c > 0 and ff[(c - 1) // 2]:
            cheb_transfer[c] = tensor_lagrange(*boxes[(c - 1) // 2], cheb, nodes[c])

    rank = np.zeros(ncl, dtype=np.int64)
    if tol <= 0.0:
        for c in boxes:
            rank[c] = big_p
        proj = {c: np.eye(big_p) for c in boxes}
        return H2Matrix(tree, bt, ff, x_tree, scale, diag, cheb, nodes, rank,
                        cheb_leaf, cheb_transfer, proj, kernel)

    # --- R1: orthogonalise bottom-up: V_t = Phi_t Z_t, Phi nested through Psi.
    z = {}
    psi_leaf = {}
    psi = {}
    for lev in range(tree.depth + 1):
        for c in tree.clusters_at_level(lev):
            if not ff[c]:
                continue
            if lev == 0:
                m = cheb_leaf[c]
            else:
                m = np.vstack([z[s] @ cheb_transfer[s] for s in (2 * c + 1, 2 * c + 2)])
            q, r = np.linalg.qr(m, mode="reduced")
            z[c] = r
            if lev == 0:
                psi_leaf[c] = q
            else:
                k1 = z[2 * c + 1].shape[0]
                psi[2 * c + 1] = q[:k1]
                psi[2 * c + 2] = q[k1:]
    # --- R2: farfield weights top-down: W_t W_t^T = sum_s D0 D0^T + Psi W_p W_p^T Psi^T.
    far_of = {c: [] for c in boxes}
    for k in range(tree.depth + 1):
        for t, s in bt.far[k]:
            far_of[int(t)].append(int(s))
    weight = {}
    for lev in range(tree.depth, -1, -1):
        for c in tree.clusters_at_level(lev):
            if not ff[c]:
                continue
            cols = [z[c] @ kernel_block(nodes[c], nodes[s], scale, kernel) @ z[s].T
                    for s in far_of[c]]
            if c > 0 and ff[(c - 1) // 2]:
                cols.append(psi[c] @ weight[(c - 1) // 2])
            wide = np.hstack(cols)
            weight[c] = _householder_r(wide.T).T
    # --- R3: truncate bottom-up.
    new_leaf = {}
    new_transfer = {}
    pi = {}
    for lev in range(tree.depth + 1):
        for c in tree.clusters_at_level(lev):
            if not ff[c]:
                continue
            if lev == 0:
                yhat = np.eye(z[c].shape[0])
            else:
                yhat = np.vstack([pi[s] @ psi[s] for s in (2 * c + 1, 2 * c + 2)])
            u, sig, _ = np.linalg.svd(yhat @ weight[c], full_matrices=False)
            keep = int(np.count_nonzero(sig > tol * sig[0])) if sig[0] > 0 else 1
            keep = max(1, keep)
            if rank_cap > 0:
                keep = min(keep, rank_cap)
            uk = u[:, :keep]
            rank[c] = keep
            pi[c] = uk.T @ yhat
            if lev == 0:
                new_leaf[c] = psi_leaf[c] @ uk
            else:
                k1 = rank[2 * c + 1]
                new_transfer[2 * c + 1] = uk[:k1]
                new_transfer[2 * c + 2] = uk[k1:]
    proj = {c: pi[c] @ z[c] for c in boxes}
    return H2Matrix(tree, bt, ff, x_tree, scale, diag, cheb, nodes, rank,
                    new_leaf, new_transfer, proj, kernel)
