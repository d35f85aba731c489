"""Pins of the oracle for the preconditioner variant of Section 5.5: the
Example 4 matrix, block threshold ILU of S and right-preconditioned GMRES.

Checks rest on what does not depend on the oracle's own formulas: values
written out by hand, scipy's pairwise distances, block ILU(0) and the dense
solve of S at the two ends of the drop tolerance, and closed-form behaviour
of GMRES (finite termination, exact preconditioner, dense solves).
"""

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import h2inputs
import oracle
from oracle import h2 as oh2


def ifmm_dense(x, d):
    r = cdist(x, x)
    with np.errstate(divide="ignore"):
        a = np.where(r < d, r / d, d / r)
    np.fill_diagonal(a, 1.0)
    return a


def test_ifmm_kernel_values_by_hand():
    """Example 4: 1 on the diagonal, r/d below d, d/r from d on."""
    d = 0.01
    x = np.array([[0.0, 0.0, 0.0], [0.005, 0.0, 0.0], [0.0, 0.0, 0.02], [0.0, 0.01, 0.0]])
    idx = np.arange(4)
    got = oh2.close_block(x, idx, idx, 1.0, 1.0, (oracle.IFMM, d))
    assert got[0, 1] == pytest.approx(0.5, abs=1e-15)
    assert got[0, 2] == pytest.approx(0.5, abs=1e-15)
    assert got[0, 3] == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.diag(got) == 1.0)
    assert np.array_equal(got, got.T)


@pytest.fixture(scope="module")
def ifmm_case():
    x = h2inputs.points("cube", 1500, 41)
    out = {}
    for d in (1e-3, 1e-2):
        fine = oracle.build_h2(x, 32, 4, 1.0, 1.0, 1e-9, 64, 1.0, (oracle.IFMM, d))
        coarse = oracle.build_h2(x, 32, 4, 1.0, 1.0, 1e-3, 64, 1.0, (oracle.IFMM, d))
        sp = oracle.sparsify(coarse)
        out[d] = (x, fine, coarse, sp, oracle.elimination_order(sp))
    return out


def test_ifmm_h2_and_conditioning(ifmm_case):
    """The H^2 of Example 4 against the dense matrix, and the paper's
    observation that the condition number grows with d."""
    cond = {}
    for d, (x, fine, coarse, sp, order) in ifmm_case.items():
        exact = ifmm_dense(fine.x_tree, d)
        assert np.linalg.norm(fine.dense() - exact) <= 1e-4 * np.linalg.norm(exact)
        cond[d] = np.linalg.cond(exact)
    assert cond[1e-2] > 100 * cond[1e-3]


def test_ilut_infinite_tolerance_is_ilu0(ifmm_case):
    x, fine, coarse, sp, order = ifmm_case[1e-2]
    il = oracle.BlockILUT(sp, np.inf, order)
    assert il.kept_fill == 0 and il.dropped > 0
    r = np.random.default_rng(3).standard_normal((sp.n, 2))
    want = oracle.BlockILU0(sp, order).solve(r)
    assert np.abs(il.solve(r) - want).max() <= 1e-12 * np.abs(want).max()


def test_ilut_zero_tolerance_is_exact(ifmm_case):
    x, fine, coarse, sp, order = ifmm_case[1e-2]
    il = oracle.BlockILUT(sp, 0.0, order)
    assert il.dropped == 0
    assert il.kept_fill == len(oracle.block_fill(sp, order)) - len(sp.s_blocks)
    r = np.random.default_rng(4).standard_normal((sp.n, 2))
    want = np.linalg.solve(oracle.dense_s(sp), r)
    assert np.abs(il.solve(r) - want).max() <= 1e-11 * np.abs(want).max()


def test_gmres_finite_termination():
    """On a diagonal matrix with k distinct eigenvalues GMRES is exact after
    at most k steps (the Krylov space holds the solution)."""
    lam = np.repeat([1.0, 2.0, 5.0, 11.0], 25)
    b = np.random.default_rng(5).standard_normal((100, 1))
    x, hist = oracle.gmres(lambda v: lam[:, None] * v, b, tol=1e-13, restart=50)
    assert len(hist[0]) <= 4
    assert np.abs(x[:, 0] - b[:, 0] / lam).max() <= 1e-12


def test_gmres_dense_solve_exact_preconditioner_and_restart():
    rng = np.random.default_rng(6)
    a = np.eye(80) * 4 + rng.standard_normal((80, 80)) / np.sqrt(80)
    b = rng.standard_normal((80, 3))
    want = np.linalg.solve(a, b)
    x, hist = oracle.gmres(lambda v: a @ v, b, tol=1e-12, restart=80)
    assert np.abs(x - want).max() <= 1e-10 * np.abs(want).max()
    ainv = np.linalg.inv(a)
    x1, hist1 = oracle.gmres(lambda v: a @ v, b, lambda v: ainv @ v, tol=1e-12)
    assert all(len(h) == 1 for h in hist1)
    assert np.abs(x1 - want).max() <= 1e-10 * np.abs(want).max()
    xr, histr = oracle.gmres(lambda v: a @ v, b, tol=1e-12, restart=4, max_iter=400)
    assert np.abs(xr - want).max() <= 1e-10 * np.abs(want).max()
    assert max(len(h) for h in histr) > 4          # it did restart


@pytest.mark.parametrize("d", [1e-3, 1e-2])
def test_gmres_with_ilut_preconditioner(ifmm_case, d):
    """Section 5.5's setup: GMRES to 1e-10 on the fine H^2 (1e-9), the
    preconditioner the sparsified coarse H^2 (1e-3) with block ILUt; the
    solution against the dense solve of the fine H^2."""
    x, fine, coarse, sp, order = ifmm_case[d]
    il = oracle.BlockILUT(sp, 1e-2, order)
    pre = lambda v: oracle.apply_v(sp, il.solve(oracle.apply_ut(sp, v)))
    b = np.random.default_rng(7).standard_normal((fine.tree.n, 2))
    xs, hist = oracle.gmres(fine.matvec, b, pre, tol=1e-10)
    assert max(len(h) for h in hist) <= 20
    assert np.max(np.linalg.norm(b - fine.matvec(xs), axis=0) / np.linalg.norm(b, axis=0)) <= 1e-10
    want = np.linalg.solve(fine.dense(), b)
    assert np.abs(xs - want).max() <= 1e-7 * np.abs(want).max()
