"""Oracle: Householder QR with a square orthogonal factor (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package.

Section 4.2 completes each (orthogonalised) cluster basis block to a square
orthogonal block by a QR decomposition with a square Q factor.  The paper
fixes no convention; the one used here is LAPACK's (dgeqrf / dlarfg /
dorgqr): reflector j maps column j onto beta * e_j with
beta = -sign(alpha) * ||(alpha, x)||, sign(alpha) = +1 for alpha >= 0,
H_j = I - tau_j v_j v_j^T with v_j(0) = 1, tau_j = 0 when x = 0, and
Q = H_0 H_1 ... H_{q-1} formed explicitly as an n x n matrix, q = min(n, r).
"""

from __future__ import annotations

import math

import numpy as np


def householder_qr(b: np.ndarray):
    """Returns (Q, R): Q (n x n) orthogonal, R (n x r) upper trapezoidal, B = Q R."""
    a = np.array(b, dtype=np.float64, copy=True)
    n, r = a.shape
    q = min(n, r)
    taus = []
    vecs = []
    for j in range(q):
        alpha = a[j, j]
        x = a[j + 1:, j]
        xnorm2 = float(np.dot(x, x))
        v = np.zeros(n - j)
        v[0] = 1.0
        if xnorm2 == 0.0:
            tau = 0.0
        else:
            norm = math.sqrt(alpha * alpha + xnorm2)
            beta = -norm if alpha >= 0.0 else norm
            tau = (beta - alpha) / beta
            v[1:] = x / (alpha - beta)
            a[j, j] = beta
            a[j + 1:, j] = 0.0
            if j + 1 < r:
                w = v @ a[j:, j + 1:]
                a[j:, j + 1:] -= tau * np.outer(v, w)
        taus.append(tau)
        vecs.append(v)
    qmat = np.eye(n)
    for j in range(q - 1, -1, -1):
        v = vecs[j]
        w = v @ qmat[j:, :]
        qmat[j:, :] -= taus[j] * np.outer(v, w)
    return qmat, a
