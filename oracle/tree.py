"""Oracle: cluster tree, block cluster tree and admissibility (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package.

Follows Section 4.1 (Definitions 4.1-4.4: row/column cluster trees, block
cluster tree, admissibility condition, farfield/nearfield sets) with the
level numbering of Section 2 (level 0 = leaves, block size doubling per
level).  Where the paper is silent the readings are:

* binary kd-tree, all leaves at the same depth L = smallest L >= 0 with
  ceil(N / 2^L) <= leaf; a cluster is split along the longest axis of its
  tight bounding box (lowest axis on ties), its points ordered by
  (coordinate, original index), the first floor(n/2) go to the left son;
* clusters are numbered in heap order (root 0, sons of c are 2c+1, 2c+2),
  so the clusters of one depth are contiguous and left-to-right;
* adm(t, s) <=> t != s and d^2 > 0 and d^2 >= eta^2 * max(diam_t^2, diam_s^2)
  on tight boxes, evaluated term by term in axis order (no fused ops);
* block cluster tree with equal-depth leaves: sons(t, s) = sons(t) x sons(s)
  (the paper's first two cases carry identical conditions).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def tree_depth(n: int, leaf: int) -> int:
    """Smallest L >= 0 with ceil(n / 2^L) <= leaf (integer arithmetic only)."""
    depth = 0
    while ((n + (1 << depth) - 1) >> depth) > leaf:
        depth += 1
    return depth


@dataclass
class ClusterTree:
    n: int
    dim: int
    depth: int                 # L: leaves sit at depth L, i.e. level 0
    perm: np.ndarray           # perm[i] = original index of tree position i
    start: np.ndarray          # per cluster (heap order) first tree position
    size: np.ndarray           # per cluster number of points
    lo: np.ndarray             # (ncl, dim) tight box lower corner
    hi: np.ndarray             # (ncl, dim) tight box upper corner

    @property
    def ncl(self) -> int:
        return (1 << (self.depth + 1)) - 1

    def level(self, c: int) -> int:
        return self.depth - (int(c + 1).bit_length() - 1)

    def clusters_at_level(self, k: int) -> np.ndarray:
        d = self.depth - k
        return np.arange((1 << d) - 1, (1 << (d + 1)) - 1)


def build_cluster_tree(x: np.ndarray, leaf: int) -> ClusterTree:
    """kd-tree on points x (n, dim); see the module docstring for the rules."""
    x = np.asarray(x, dtype=np.float64)
    n, dim = x.shape
    depth = tree_depth(n, leaf)
    ncl = (1 << (depth + 1)) - 1
    start = np.zeros(ncl, dtype=np.int64)
    size = np.zeros(ncl, dtype=np.int64)
    lo = np.zeros((ncl, dim))
    hi = np.zeros((ncl, dim))
    order = np.arange(n, dtype=np.int64)
    start[0], size[0] = 0, n
    for c in range(ncl):
        s0, sz = start[c], size[c]
        idx = order[s0:s0 + sz]
        pts = x[idx]
        lo[c] = pts.min(axis=0)
        hi[c] = pts.max(axis=0)
        if 2 * c + 1 >= ncl:
            continue
        axis = int(np.argmax(hi[c] - lo[c]))
        srt = np.lexsort((idx, pts[:, axis]))
        order[s0:s0 + sz] = idx[srt]
        nl = sz // 2
        start[2 * c + 1], size[2 * c + 1] = s0, nl
        start[2 * c + 2], size[2 * c + 2] = s0 + nl, sz - nl
    return ClusterTree(n, dim, depth, order, start, size, lo, hi)


def admissible(tree: ClusterTree, t: np.ndarray, s: np.ndarray, eta: float = 1.0) -> np.ndarray:
    """Vectorised admissibility predicate over pairs (t[i], s[i]).

    ``eta = 0`` selects weak admissibility (every pair t != s is admissible),
    the HODLR special case of the remark closing Section 2.
    """
    if eta == 0.0:
        return t != s
    d2 = np.zeros(t.shape[0])
    dt2 = np.zeros(t.shape[0])
    ds2 = np.zeros(t.shape[0])
    for a in range(tree.dim):
        gap = np.maximum(0.0, np.maximum(tree.lo[s, a] - tree.hi[t, a],
                                         tree.lo[t, a] - tree.hi[s, a]))
        d2 = d2 + gap * gap
        et = tree.hi[t, a] - tree.lo[t, a]
        es = tree.hi[s, a] - tree.lo[s, a]
        dt2 = dt2 + et * et
        ds2 = ds2 + es * es
    bound = np.maximum(dt2, ds2) * (eta * eta)
    return (t != s) & (d2 > 0.0) & (d2 >= bound)


@dataclass
class BlockTree:
    """Per level k: near[k] (inadmissible pairs, N_k) and far[k] (I_k)."""
    near: list = field(default_factory=list)
    far: list = field(default_factory=list)


def build_block_tree(tree: ClusterTree, eta: float = 1.0) -> BlockTree:
    """Recursive subdivision from (root, root); Definitions 4.2-4.4.

    Pairs are kept sorted lexicographically by (t, s) at every level.
    """
    depth = tree.depth
    near = [None] * (depth + 1)
    far = [None] * (depth + 1)
    cur = np.array([[0, 0]], dtype=np.int64)
    for k in range(depth, -1, -1):
        adm = admissible(tree, cur[:, 0], cur[:, 1], eta)
        f = cur[adm]
        nr = cur[~adm]
        far[k] = f[np.lexsort((f[:, 1], f[:, 0]))]
        near[k] = nr[np.lexsort((nr[:, 1], nr[:, 0]))]
        if k > 0:
            t, s = near[k][:, 0], near[k][:, 1]
            kids = []
            for a in (1, 2):
                for b in (1, 2):
                    kids.append(np.stack([2 * t + a, 2 * s + b], axis=1))
            cur = np.concatenate(kids, axis=0) if kids else np.zeros((0, 2), np.int64)
    return BlockTree(near, far)


def farfield_nonempty(tree: ClusterTree, bt: BlockTree) -> np.ndarray:
    """ff[t] is True iff t or one of its ancestors has an admissible pair."""
    ff = np.zeros(tree.ncl, dtype=bool)
    for k in range(tree.depth + 1):
        if bt.far[k].shape[0]:
            ff[bt.far[k][:, 0]] = True
    for c in range(1, tree.ncl):
        ff[c] |= ff[(c - 1) // 2]
    return ff
