"""Oracle: the preconditioner variant of Section 5.5 (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package.

Section 5.5 solves A x = b by GMRES on the H^2 matrix-vector product, with
the sparsification of a coarser H^2 approximation of A, factorised
incompletely by ILUt, as the preconditioner.  The paper names ILUt and its
drop tolerance tau but not the variant; the reading used here is a block
form of the threshold ILU:

* block rows are eliminated in an elimination order (IKJ form), each row
  over the structural fill of exact elimination;
* a block of the factor outside S's own pattern (fill) is dropped when its
  Frobenius norm is below tau times the Frobenius norm of block row i of S
  as given: an L-part block right after it is scaled by the pivot (before
  it updates anything), a U-part block when its row is finished;
* blocks of S's own pattern are never dropped.

So tau = infinity is block ILU(0) and tau = 0 is the exact block
factorisation; both are pinned.  GMRES is the textbook method: right
preconditioned (the residual monitored is that of A x = b), Arnoldi by
modified Gram-Schmidt, the small least-squares problem by Givens rotations,
restarted every ``restart`` steps, column by column.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .sparsify import Sparsified


class BlockILUT:
    """Block threshold ILU of S (IKJ form) in S order or a given elimination order."""

    def __init__(self, sp: Sparsified, tau: float, order=None):
        self.sp = sp
        if order is None:
            order = sp.order
        order = [int(c) for c in order if sp.nonbasis[c] > 0]
        self.order = order
        self.pos = {c: i for i, c in enumerate(order)}
        pattern = {c: set() for c in order}
        for (t, s) in sp.s_blocks:
            pattern[t].add(s)
        ref = {c: 0.0 for c in order}
        for (t, s), blk in sp.s_blocks.items():
            ref[t] += float(np.sum(blk * blk))
        ref = {c: np.sqrt(v) for c, v in ref.items()}
        self.upper = {}       # i -> {j: U_ij} for j after i (j == i: the pivot block)
        self.lower = {}       # i -> {k: L_ik} for k before i
        self.piv = {}
        self.dropped = 0
        self.kept_fill = 0
        for i in order:
            pi = self.pos[i]
            w = {j: sp.s_blocks[(i, j)].copy() for j in pattern[i]}
            low = {}
            done = set()
            while True:
                # next block of row i before the diagonal, in elimination order
                ks = [k for k in w if self.pos[k] < pi and k not in done]
                if not ks:
                    break
                k = min(ks, key=lambda u: self.pos[u])
                done.add(k)
                lik = sla.lu_solve(self.piv[k], w.pop(k).T, trans=1).T
                if k not in pattern[i] and np.linalg.norm(lik) < tau * ref[i]:
                    self.dropped += 1
                    continue
                if k not in pattern[i]:
                    self.kept_fill += 1
                low[k] = lik
                for j, ukj in self.upper[k].items():
                    if j == k:
                        continue
                    if j not in w:
                        w[j] = np.zeros((sp.nonbasis[i], sp.nonbasis[j]))
                    w[j] -= lik @ ukj
            up = {}
            for j, blk in w.items():
                if j != i and j not in pattern[i] and np.linalg.norm(blk) < tau * ref[i]:
                    self.dropped += 1
                    continue
                if j != i and j not in pattern[i]:
                    self.kept_fill += 1
                up[j] = blk
            self.piv[i] = sla.lu_factor(up[i])
            self.upper[i] = up
            self.lower[i] = low

    def solve(self, r_s: np.ndarray) -> np.ndarray:
        """(L U)^{-1} r for r in S order (n, nrhs)."""
        sp = self.sp
        r = r_s.reshape(sp.n, -1)

        def rows_of(c):
            return slice(sp.soff[c], sp.soff[c] + sp.nonbasis[c])

        y = np.zeros_like(r)
        for i in self.order:
            acc = r[rows_of(i)].copy()
            for k, lik in self.lower[i].items():
                acc -= lik @ y[rows_of(k)]
            y[rows_of(i)] = acc
        x = np.zeros_like(r)
        for i in reversed(self.order):
            acc = y[rows_of(i)].copy()
            for j, uij in self.upper[i].items():
                if j != i:
                    acc -= uij @ x[rows_of(j)]
            x[rows_of(i)] = sla.lu_solve(self.piv[i], acc)
        return x.reshape(r_s.shape)


class SymBlockILUT:
    """Symmetric block threshold incomplete factorisation S ~ U^T D^{-1} U
    (block L D L^T with L_ik = U_ki^T D_k^{-1}, D_i = U_ii) in an
    elimination order: the reading of ILUt for a symmetric S (Proposition
    2.1), whose factor stays symmetric.

    Row i, left-looking: its blocks at or after i in the order start as S_ij;
    every earlier row k whose block (k, i) was kept subtracts
    U_ki^T D_k^{-1} U_kj from block (i, j) for each kept U_kj with j at or
    after i (a fill block where S_ij is not stored).  Once row i is finished,
    a fill block (i, j), j after i, is dropped when its Frobenius norm is
    below tau times that of block row i of S as given (both triangles);
    blocks of S's own pattern are kept.  The drop decision is taken once, on
    the upper block; the lower block L_ji mirrors it.  tau = infinity keeps
    S's pattern (block ILU(0)), tau = 0 the whole structural fill (the exact
    factorisation).
    """

    def __init__(self, sp: Sparsified, tau: float, order=None):
        self.sp = sp
        if order is None:
            order = sp.order
        order = [int(c) for c in order if sp.nonbasis[c] > 0]
        self.order = order
        self.pos = pos = {c: i for i, c in enumerate(order)}
        upat = {c: set() for c in order}
        ref = {c: 0.0 for c in order}
        for (t, u), blk in sp.s_blocks.items():
            ref[t] += float(np.sum(blk * blk))
            if pos[u] >= pos[t]:
                upat[t].add(u)
        ref = {c: np.sqrt(v) for c, v in ref.items()}
        self.upper = {}          # i -> {j: U_ij}, j at or after i
        self.piv = {}            # i -> LU of D_i = U_ii
        above = {c: [] for c in order}   # j -> rows k before j with U_kj kept
        self.dropped = 0
        self.kept_fill = 0
        for i in order:
            w = {j: sp.s_blocks[(i, j)].copy() for j in upat[i]}
            for k in sorted(above[i], key=lambda u: pos[u]):
                zki = sla.lu_solve(self.piv[k], self.upper[k][i])      # D_k^{-1} U_ki
                for j, ukj in self.upper[k].items():
                    if pos[j] < pos[i]:
                        continue
                    upd = zki.T @ ukj
                    w[j] = w[j] - upd if j in w else -upd
            up = {}
            for j, blk in w.items():
                if j != i and j not in upat[i]:
                    if np.linalg.norm(blk) < tau * ref[i]:
                        self.dropped += 1
                        continue
                    self.kept_fill += 1
                up[j] = blk
            self.piv[i] = sla.lu_factor(up[i])
            self.upper[i] = up
            for j in up:
                if j != i:
                    above[j].append(i)

    def solve(self, r_s: np.ndarray) -> np.ndarray:
        """(U^T D^{-1} U)^{-1} r for r in S order (n, nrhs)."""
        sp = self.sp
        r = r_s.reshape(sp.n, -1)

        def rows_of(c):
            return slice(sp.soff[c], sp.soff[c] + sp.nonbasis[c])

        z = r.copy()
        for k in self.order:                       # z = L^{-1} r
            dz = sla.lu_solve(self.piv[k], z[rows_of(k)])
            for j, ukj in self.upper[k].items():
                if j != k:
                    z[rows_of(j)] -= ukj.T @ dz
        x = np.zeros_like(r)
        for i in reversed(self.order):             # x = D^{-1} L^{-T}-part
            acc = z[rows_of(i)].copy()
            for j, uij in self.upper[i].items():
                if j != i:
                    acc -= uij @ x[rows_of(j)]
            x[rows_of(i)] = sla.lu_solve(self.piv[i], acc)
        return x.reshape(r_s.shape)


def gmres(matvec, b: np.ndarray, precond=None, tol: float = 1e-10, restart: int = 50,
          max_iter: int = 500):
    """Right-preconditioned restarted GMRES, column by column.

    Solves A x = b with A = matvec and M^{-1} = precond (identity if None):
    GMRES on A M^{-1} u = b, x = M^{-1} u.  Stops when ||b - A x|| <=
    tol ||b|| (the small problem's residual estimate, confirmed by a true
    residual at every restart and at the end).  Returns x and, per column,
    the list of relative residual estimates after every Arnoldi step.
    """
    b = b.reshape(b.shape[0], -1)
    x = np.zeros_like(b)
    histories = []
    apply_m = precond if precond is not None else (lambda v: v)
    for col in range(b.shape[1]):
        bj = b[:, col]
        bn = np.linalg.norm(bj)
        xj = np.zeros_like(bj)
        hist = []
        steps = 0
        if bn == 0.0:
            histories.append(hist)
            continue
        while steps < max_iter:
            r = bj - matvec(xj[:, None])[:, 0]
            beta = np.linalg.norm(r)
            if beta <= tol * bn:
                break
            m = min(restart, max_iter - steps)
            v = np.zeros((bj.shape[0], m + 1))
            z = np.zeros((bj.shape[0], m))
            h = np.zeros((m + 1, m))
            cs = np.zeros(m)
            sn = np.zeros(m)
            g = np.zeros(m + 1)
            g[0] = beta
            v[:, 0] = r / beta
            used = 0
            for j in range(m):
                z[:, j] = apply_m(v[:, j:j + 1])[:, 0]
                wv = matvec(z[:, j:j + 1])[:, 0]
                for i in range(j + 1):                 # modified Gram-Schmidt
                    h[i, j] = wv @ v[:, i]
                    wv = wv - h[i, j] * v[:, i]
                h[j + 1, j] = np.linalg.norm(wv)
                if h[j + 1, j] > 0.0:
                    v[:, j + 1] = wv / h[j + 1, j]
                for i in range(j):                     # earlier rotations
                    t = cs[i] * h[i, j] + sn[i] * h[i + 1, j]
                    h[i + 1, j] = -sn[i] * h[i, j] + cs[i] * h[i + 1, j]
                    h[i, j] = t
                rho = np.hypot(h[j, j], h[j + 1, j])   # new rotation zeroes h[j+1, j]
                cs[j], sn[j] = h[j, j] / rho, h[j + 1, j] / rho
                h[j, j] = rho
                h[j + 1, j] = 0.0
                g[j + 1] = -sn[j] * g[j]
                g[j] = cs[j] * g[j]
                used = j + 1
                steps += 1
                hist.append(abs(g[j + 1]) / bn)
                if abs(g[j + 1]) <= tol * bn or h[j, j] == 0.0:
                    break
            yk = sla.solve_triangular(h[:used, :used], g[:used])
            xj = xj + z[:, :used] @ yk
        x[:, col] = xj
        histories.append(hist)
    return x, histories
