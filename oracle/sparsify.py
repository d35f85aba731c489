"""Oracle: non-extensive sparsification A = U S V^T of an H^2 matrix (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package.

Follows Section 2 (compression at level zero, at the first level and at all
levels; the equations for U_0^T A V_0, the permuted close matrix and the new
close matrix C_1, the extended U_1 / V_1 and the final A = U S V^T) in the
form Section 4 gives it for H^2 coefficients (4.2: U, V from the cluster
bases completed by QR with a square Q; 4.3: S from the close matrix and the
couplings of the interaction lists).  Readings where the paper is loose:

* per-cluster sizes: n_t = |t| at a leaf, else the sum of the sons' kept
  rows; k_t = min(n_t, r_t) rows are passed up when t (or an ancestor) has
  a farfield, otherwise k_t = 0; m_t = n_t - k_t rows are finalised in S;
* "close" at level k >= 1 is H^2 inadmissibility: for (t, s) in N_k the
  block C_k(t, s) is made of X_{k-1}(a, b)[:k_a, :k_b] for son pairs in
  N_{k-1} and R^_a D_ab R^_b^T for son pairs in I_{k-1};
* basis rows come first inside a cluster after Q_t^T; S orders the
  non-basis rows level by level from the leaves up, clusters left to
  right, each cluster's rows in Q column order k_t .. n_t - 1;
* finalised rows (columns) keep receiving the column (row) transforms of the
  higher levels: these are the off-level blocks S_ij of Section 3.

The general (row and column) algorithm is carried out; the symmetry of S
for a symmetric H^2 matrix (Proposition 2.1) is a property tested on it.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .h2 import H2Matrix, close_block
from .householder import householder_qr


@dataclass
class Sparsified:
    h2: H2Matrix
    n_act: np.ndarray       # n_t
    kept: np.ndarray        # k_t
    nonbasis: np.ndarray    # m_t
    soff: np.ndarray        # first S row of cluster t
    order: np.ndarray       # clusters in S order
    q: dict                 # t -> Q_t (n_t x n_t)
    rhat: dict              # t -> R^_t (k_t x r_t)
    s_blocks: dict          # (t, s) -> S block (m_t x m_s)

    @property
    def n(self) -> int:
        return self.h2.tree.n


def cluster_sizes(h2: H2Matrix):
    """n_t, k_t, m_t per cluster (heap order), bottom-up."""
    tr = h2.tree
    n_act = np.zeros(tr.ncl, dtype=np.int64)
    kept = np.zeros(tr.ncl, dtype=np.int64)
    for lev in range(tr.depth + 1):
        for c in tr.clusters_at_level(lev):
            if lev == 0:
                n_act[c] = tr.size[c]
            else:
                n_act[c] = kept[2 * c + 1] + kept[2 * c + 2]
            kept[c] = min(n_act[c], h2.rank[c]) if h2.ff[c] else 0
    return n_act, kept, n_act - kept


def s_order(h2: H2Matrix, nonbasis: np.ndarray):
    """Clusters in S order (level 0 first, left to right) and their S offsets."""
    tr = h2.tree
    order = np.concatenate([tr.clusters_at_level(lev) for lev in range(tr.depth + 1)])
    soff = np.zeros(tr.ncl, dtype=np.int64)
    pos = 0
    for c in order:
        soff[c] = pos
        pos += nonbasis[c]
    assert pos == tr.n
    return order, soff


def sparsify(h2: H2Matrix) -> Sparsified:
    tr = h2.tree
    n_act, kept, nonbasis = cluster_sizes(h2)
    order, soff = s_order(h2, nonbasis)
    idx = np.arange(tr.n)

    def son_offset(c: int) -> int:
        """Row offset of son c inside its father's active rows."""
        return 0 if c % 2 == 1 else int(kept[c - 1])

    qs, rhat, s_blocks = {}, {}, {}
    prev_x = {}                       # X_{k-1}(t, s) of the previous level
    row_carry, col_carry = {}, {}     # strip remainders passed to the next level
    near_prev = set()
    far_prev = []
    for lev in range(tr.depth + 1):
        clusters = tr.clusters_at_level(lev)
        # --- basis completion: B_t = Q_t [R^_t; 0]  (Section 4.2)
        for t in clusters:
            if n_act[t] == 0:
                continue
            if kept[t] == 0:
                qs[t] = np.eye(n_act[t])
                continue
            if lev == 0:
                b = h2.leaf_basis[t]
            else:
                b = np.vstack([rhat[c] @ h2.transfer[c] for c in (2 * t + 1, 2 * t + 2)
                               if kept[c] > 0])
            qmat, r = householder_qr(b)
            qs[t] = qmat
            rhat[t] = r[:kept[t]]
        # --- close blocks C_lev(t, s) and their two-sided transform
        cur_x = {}
        for t, s in h2.bt.near[lev]:
            t, s = int(t), int(s)
            if n_act[t] == 0 or n_act[s] == 0:
                continue
            if lev == 0:
                ts, ss = h2.cluster_slice(t), h2.cluster_slice(s)
                c = close_block(h2.x_tree, idx[ts], idx[ss], h2.scale, h2.diag, h2.kernel)
            else:
                c = np.zeros((n_act[t], n_act[s]))
                for a in (2 * t + 1, 2 * t + 2):
                    for b in (2 * s + 1, 2 * s + 2):
                        ka, kb = kept[a], kept[b]
                        if ka == 0 or kb == 0:
                            continue
                        oa, ob = son_offset(a), son_offset(b)
                        if (a, b) in near_prev:
                            piece = prev_x[(a, b)][:ka, :kb]
                        else:
                            piece = rhat[a] @ h2.coupling(a, b) @ rhat[b].T
                        c[oa:oa + ka, ob:ob + kb] = piece
            x = qs[t].T @ c @ qs[s]
            cur_x[(t, s)] = x
            kt, ks = kept[t], kept[s]
            if nonbasis[t] > 0 and nonbasis[s] > 0:
                s_blocks[(t, s)] = x[kt:, ks:].copy()
        # --- strips: finalised rows/columns receive this level's transforms
        row_in, col_in = {}, {}
        for (tau, c), piece in row_carry.items():
            row_in.setdefault((tau, (c - 1) // 2), {})[c] = piece
        for (c, tau), piece in col_carry.items():
            col_in.setdefault(((c - 1) // 2, tau), {})[c] = piece
        if lev > 0:
            for (a, b), xprev in prev_x.items():
                ka, kb = kept[a], kept[b]
                if nonbasis[a] > 0 and kb > 0:
                    row_in.setdefault((a, (b - 1) // 2), {})[b] = xprev[ka:, :kb]
                if ka > 0 and nonbasis[b] > 0:
                    col_in.setdefault(((a - 1) // 2, b), {})[a] = xprev[:ka, kb:]
        row_carry, col_carry = {}, {}
        for (tau, p), pieces in row_in.items():
            g = np.zeros((nonbasis[tau], n_act[p]))
            for c, piece in pieces.items():
                oc = son_offset(c)
                g[:, oc:oc + kept[c]] = piece
            y = g @ qs[p]
            if nonbasis[p] > 0:
                s_blocks[(tau, p)] = y[:, kept[p]:].copy()
            if kept[p] > 0 and p > 0:
                row_carry[(tau, p)] = y[:, :kept[p]].copy()
        for (p, tau), pieces in col_in.items():
            h = np.zeros((n_act[p], nonbasis[tau]))
            for c, piece in pieces.items():
                oc = son_offset(c)
                h[oc:oc + kept[c], :] = piece
            z = qs[p].T @ h
            if nonbasis[p] > 0:
                s_blocks[(p, tau)] = z[kept[p]:, :].copy()
            if kept[p] > 0 and p > 0:
                col_carry[(p, tau)] = z[:kept[p], :].copy()
        prev_x = cur_x
        near_prev = {(int(a), int(b)) for a, b in h2.bt.near[lev]}
        far_prev = h2.bt.far[lev]
    del far_prev
    return Sparsified(h2, n_act, kept, nonbasis, soff, order, qs, rhat, s_blocks)


# ---------------------------------------------------------------- U and V (eq. sp0)

def apply_ut(sp: Sparsified, b_tree: np.ndarray) -> np.ndarray:
    """y = U^T b: leaves to root, w = Q_t^T z_t, non-basis part to y, rest upward."""
    h2, tr = sp.h2, sp.h2.tree
    b = b_tree.reshape(tr.n, -1)
    y = np.zeros_like(b)
    z = {}
    for lev in range(tr.depth + 1):
        for t in tr.clusters_at_level(lev):
            if sp.n_act[t] == 0:
                continue
            if lev == 0:
                zt = b[h2.cluster_slice(t)]
            else:
                zt = np.vstack([z.pop(c) for c in (2 * t + 1, 2 * t + 2) if sp.kept[c] > 0])
            w = sp.q[t].T @ zt
            k = sp.kept[t]
            y[sp.soff[t]:sp.soff[t] + sp.nonbasis[t]] = w[k:]
            if k > 0:
                z[t] = w[:k]
    return y.reshape(b_tree.shape)


def apply_v(sp: Sparsified, y_s: np.ndarray) -> np.ndarray:
    """x = V y: root to leaves, z_t = Q_t [z_t^basis; y_t], split to the sons."""
    h2, tr = sp.h2, sp.h2.tree
    y = y_s.reshape(tr.n, -1)
    x = np.zeros_like(y)
    z = {}
    for lev in range(tr.depth, -1, -1):
        for t in tr.clusters_at_level(lev):
            if sp.n_act[t] == 0:
                continue
            top = z.pop(t) if sp.kept[t] > 0 else np.zeros((0, y.shape[1]))
            w = np.vstack([top, y[sp.soff[t]:sp.soff[t] + sp.nonbasis[t]]])
            zt = sp.q[t] @ w
            if lev == 0:
                x[h2.cluster_slice(t)] = zt
            else:
                off = 0
                for c in (2 * t + 1, 2 * t + 2):
                    kc = sp.kept[c]
                    if kc > 0:
                        z[c] = zt[off:off + kc]
                        off += kc
    return x.reshape(y_s.shape)


def dense_s(sp: Sparsified) -> np.ndarray:
    """S as a dense N x N matrix in S order (small N only)."""
    s = np.zeros((sp.n, sp.n))
    for (t, u), blk in sp.s_blocks.items():
        s[sp.soff[t]:sp.soff[t] + sp.nonbasis[t], sp.soff[u]:sp.soff[u] + sp.nonbasis[u]] = blk
    return s


def dense_u(sp: Sparsified) -> np.ndarray:
    """U (= V for the symmetric H^2 matrix) as a dense matrix: U = V(I)."""
    return apply_v(sp, np.eye(sp.n))


def pattern_predicate(sp: Sparsified):
    """Block pattern of S from the block tree alone (the bit-exact contract).

    (t, s) with lev(t) <= lev(s), both with m > 0, is present iff some s'
    (s itself or a descendant of s on t's level) has (t, s') in N_lev(t) and
    every cluster strictly between s' and s on the path passes rows up
    (k > 0); the lower part is the transpose.
    """
    h2, tr = sp.h2, sp.h2.tree
    out = set()
    for lev in range(tr.depth + 1):
        for t, s in h2.bt.near[lev]:
            t, s = int(t), int(s)
            if sp.nonbasis[t] == 0:
                continue
            c = s
            while True:
                if sp.nonbasis[c] > 0:
                    out.add((t, c))
                    out.add((c, t))
                if c == 0 or sp.kept[c] == 0:
                    break
                c = (c - 1) // 2
    return out
