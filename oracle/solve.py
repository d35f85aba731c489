"""Oracle: solving A x = b through S y = U^T b, x = V y (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package.

Equation (sp0) of the introduction: once A = U S V^T, the system A x = b is
replaced by S y = U^T b and x = V y, S being handled by sparse tools (a
sparse direct factorisation in Section 5.3-5.4, an incomplete factorisation
used as a preconditioner in Section 5.5).  Readings used here:

* the sparse factorisation is a block LU of S in S order restricted to the
  block pattern of S (block ILU(0)): for every block row i, for every k < i
  in row i (ascending), S_ik <- S_ik S_kk^{-1}, then S_ij -= S_ik S_kj for
  every j > k in both rows; pivot blocks are handled by LU with partial
  pivoting inside the block;
* the residual is max over columns of ||b - A_H2 x||_2 / ||b||_2 with the
  H^2 matrix-vector product, and iterative refinement repeats
  x += V (LU_S)^{-1} U^T r until it drops below the tolerance.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .sparsify import Sparsified, apply_ut, apply_v, dense_s


class BlockILU0:
    """Block ILU(0) of S in S order (IKJ form)."""

    def __init__(self, sp: Sparsified):
        self.sp = sp
        order = [int(c) for c in sp.order if sp.nonbasis[c] > 0]
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
