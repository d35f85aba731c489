"""Oracle: solving A x = b through S y = U^T b, x = V y (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package.

Equation (sp0) of the introduction: once A = U S V^T, the system A x = b is
replaced by S y = U^T b and x = V y, S being handled by sparse tools (a
sparse direct factorisation in Section 5.3-5.4, an incomplete factorisation
used as a preconditioner in Section 5.5).  Readings used here:

* the sparse factorisation is a block LU of S restricted to the block
  pattern of S (block ILU(0)) in an elimination order: for every block row
  i, for every k before i in row i (in that order), S_ik <- S_ik S_kk^{-1},
  then S_ij -= S_ik S_kj for every j after k in both rows; pivot blocks are
  handled by LU with partial pivoting inside the block;
* the elimination order (a sparse solver's own choice, as CHOLMOD's
  reordering is in Section 5.3) is S order by default, or the multicolour
  order of ``elimination_order``: tree levels from the leaves up and, inside
  a level, clusters sorted by (greedy colour, index) where the colour of a
  cluster is the smallest one not taken by an earlier close neighbour on its
  level (rows of one colour share no block of S);
* the residual is max over columns of ||b - A_H2 x||_2 / ||b||_2 with the
  H^2 matrix-vector product, and iterative refinement repeats
  x += V (LU_S)^{-1} U^T r until it drops below the tolerance.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .sparsify import Sparsified, apply_ut, apply_v, dense_s


def elimination_colours(sp: Sparsified):
    """Greedy colour of every cluster with m > 0 among its close neighbours on its level."""
    tr = sp.h2.tree
    colour = {}
    for lev in range(tr.depth + 1):
        nbrs = {}
        for t, s in sp.h2.bt.near[lev]:
            t, s = int(t), int(s)
            if t != s and sp.nonbasis[t] > 0 and sp.nonbasis[s] > 0:
                nbrs.setdefault(t, []).append(s)
        for t in tr.clusters_at_level(lev):
            t = int(t)
            if sp.nonbasis[t] == 0:
                continue
            taken = {colour[s] for s in nbrs.get(t, []) if s < t}
            c = 0
            while c in taken:
                c += 1
            colour[t] = c
    return colour


def elimination_order(sp: Sparsified):
    """Multicolour elimination order: level by level, (greedy colour, cluster)."""
    tr = sp.h2.tree
    colour = elimination_colours(sp)
    return sorted(colour, key=lambda u: (tr.level(u), colour[u], u))


def block_fill(sp: Sparsified, order):
    """Block pattern of the exact factorisation of S in ``order``: graph
    elimination on the symmetric block pattern (eliminating k joins every
    pair of its later neighbours), the fill of a sparse direct factorisation
    (Sections 5.3-5.4).  Returns the set of (t, s) blocks, both orientations."""
    order = [int(c) for c in order if sp.nonbasis[c] > 0]
    pos = {c: i for i, c in enumerate(order)}
    nbr = {c: set() for c in order}
    for (t, s) in sp.s_blocks:
        if t != s:
            nbr[t].add(s)
    for k in order:
        later = [j for j in nbr[k] if pos[j] > pos[k]]
        for a in later:
            for b in later:
                if a != b:
                    nbr[a].add(b)
    out = {(c, c) for c in order}
    for t, ns in nbr.items():
        for s in ns:
            out.add((t, s))
    return out


def filled(sp: Sparsified, order):
    """A copy of ``sp`` whose S carries explicit zero blocks on the fill of
    ``block_fill``; BlockILU0 on it is the exact block factorisation."""
    import copy
    out = copy.copy(sp)
    blocks = dict(sp.s_blocks)
    for (t, s) in block_fill(sp, order):
        if (t, s) not in blocks:
            blocks[(t, s)] = np.zeros((sp.nonbasis[t], sp.nonbasis[s]))
    out.s_blocks = blocks
    return out


class BlockILU0:
    """Block ILU(0) of S (IKJ form) in S order or in a given elimination order."""

    def __init__(self, sp: Sparsified, order=None):
        self.sp = sp
        if order is None:
            order = sp.order
        order = [int(c) for c in order if sp.nonbasis[c] > 0]
        self.order = order
        self.pos = {c: i for i, c in enumerate(order)}
        rows = {c: [] for c in order}
        for (t, s) in sp.s_blocks:
            rows[t].append(s)
        self.rows = {c: sorted(v, key=lambda u: self.pos[u]) for c, v in rows.items()}
        blk = {key: val.copy() for key, val in sp.s_blocks.items()}
        self.piv = {}
        for i in order:
            pi = self.pos[i]
            row = self.rows[i]
            for k in row:
                if self.pos[k] >= pi:
                    break
                # L_ik = S_ik S_kk^{-1}
                blk[(i, k)] = sla.lu_solve(self.piv[k], blk[(i, k)].T, trans=1).T
                for j in row:
                    if self.pos[j] > self.pos[k] and (k, j) in blk:
                        blk[(i, j)] -= blk[(i, k)] @ blk[(k, j)]
            self.piv[i] = sla.lu_factor(blk[(i, i)])
        self.blk = blk

    def solve(self, r_s: np.ndarray) -> np.ndarray:
        """(L U)^{-1} r for r in S order (n, nrhs)."""
        sp = self.sp
        r = r_s.reshape(sp.n, -1)
        y = np.zeros_like(r)

        def rows_of(c):
            return slice(sp.soff[c], sp.soff[c] + sp.nonbasis[c])

        for i in self.order:
            acc = r[rows_of(i)].copy()
            for k in self.rows[i]:
                if self.pos[k] >= self.pos[i]:
                    break
                acc -= self.blk[(i, k)] @ y[rows_of(k)]
            y[rows_of(i)] = acc
        x = np.zeros_like(r)
        for i in reversed(self.order):
            acc = y[rows_of(i)].copy()
            for j in self.rows[i]:
                if self.pos[j] > self.pos[i]:
                    acc -= self.blk[(i, j)] @ x[rows_of(j)]
            x[rows_of(i)] = sla.lu_solve(self.piv[i], acc)
        return x.reshape(r_s.shape)


def dense_lu_solver(sp: Sparsified):
    """Exact LU of S (dense, small N): returns a function r -> S^{-1} r."""
    lu = sla.lu_factor(dense_s(sp))
    return lambda r: sla.lu_solve(lu, r)


def rel_residual(sp: Sparsified, b_tree: np.ndarray, x_tree: np.ndarray) -> np.ndarray:
    b = b_tree.reshape(sp.n, -1)
    r = b - sp.h2.matvec(x_tree.reshape(sp.n, -1))
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)


def refine(sp: Sparsified, s_solve, b_tree: np.ndarray, tol: float, max_iter: int = 30):
    """x += V S^{-1} U^T r until max_col ||r|| / ||b|| <= tol (tree order)."""
    b = b_tree.reshape(sp.n, -1)
    x = np.zeros_like(b)
    r = b.copy()
    history = []
    bn = np.linalg.norm(b, axis=0)
    for _ in range(max_iter):
        x = x + apply_v(sp, s_solve(apply_ut(sp, r)))
        r = b - sp.h2.matvec(x)
        res = float(np.max(np.linalg.norm(r, axis=0) / bn))
        history.append(res)
        if res <= tol:
            break
    return x.reshape(b_tree.shape), history


def conjugate_gradient(matvec, b: np.ndarray, tol: float = 1e-13, max_iter: int = 500):
    """Plain CG column by column on an SPD operator (reference solution)."""
    b = b.reshape(b.shape[0], -1)
    x = np.zeros_like(b)
    for j in range(b.shape[1]):
        bj = b[:, j]
        xj = np.zeros_like(bj)
        r = bj.copy()
        p = r.copy()
        rr = r @ r
        bn = np.sqrt(bj @ bj)
        for _ in range(max_iter):
            ap = matvec(p[:, None])[:, 0]
            alpha = rr / (p @ ap)
            xj += alpha * p
            r -= alpha * ap
            rr_new = r @ r
            if np.sqrt(rr_new) <= tol * bn:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        x[:, j] = xj
    return x
