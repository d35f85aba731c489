"""Shared helpers of the test suite (tests may call the oracle; the product never does)."""

import numpy as np

import h2inputs
import oracle


def kernel_scale(x):
    n = x.shape[0]
    return 1.0 / n if x.shape[1] == 2 else 1.0 / (4.0 * np.pi * n)


def make_case(kind, n, seed, leaf, cheb, tol=0.0, cap=0, eta=1.0):
    x = h2inputs.points(kind, n, seed)
    sc = kernel_scale(x)
    h2 = oracle.build_h2(x, leaf, cheb, sc, 1.0, tol, cap, eta)
    return x, sc, h2


def import_arrays(h2):
    """The oracle's H^2 coefficients in the layout of h2_import."""
    tr = h2.tree
    ncl = tr.ncl
    big_p = h2.cheb ** tr.dim
    rank = h2.rank.astype(np.int32)
    nodes = np.zeros((ncl, big_p, tr.dim))
    proj, basis, transfer = [], [], []
    for c in range(ncl):
        if not h2.ff[c]:
            continue
        nodes[c] = h2.nodes[c]
        proj.append(np.asarray(h2.proj[c]).ravel(order="F"))
        if 2 * c + 1 >= ncl:
            basis.append(np.asarray(h2.leaf_basis[c]).ravel(order="F"))
        if c > 0 and h2.ff[(c - 1) // 2]:
            transfer.append(np.asarray(h2.transfer[c]).ravel(order="F"))
    cat = lambda lst: np.concatenate(lst) if lst else np.zeros(0)
    return rank, nodes.ravel(), cat(proj), cat(basis), cat(transfer)
