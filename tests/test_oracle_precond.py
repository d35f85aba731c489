"""Pins of the oracle for the preconditioner variant of Section 5.5: the
Example 5.4 matrix, block threshold ILU of S and right-preconditioned GMRES.

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
    """Example 5.4: 1 on the diagonal, r/d below d, d/r from d on."""
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
    """The H^2 of Example 5.4 against the dense matrix, and the paper's
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


def _dense_sym_ilut(sp, tau, order):
    """Brute force of the symmetric threshold factorisation on the dense S:
    right-looking (every finished row updates the whole trailing matrix at
    once), the drop rule applied to the upper blocks of a row when its turn
    comes, mirrored onto the lower blocks.  Returns the solver of
    U^T D^{-1} U built from the finished rows."""
    sl = {c: slice(sp.soff[c], sp.soff[c] + sp.nonbasis[c]) for c in order}
    pos = {c: i for i, c in enumerate(order)}
    a = oracle.dense_s(sp)
    ref = {c: np.linalg.norm(a[sl[c], :]) for c in order}
    own = set(sp.s_blocks)
    u_rows = {}
    for k in order:
        later = [j for j in order if pos[j] > pos[k]]
        for j in later:
            blk = a[sl[k], sl[j]]
            if (k, j) not in own and np.any(blk != 0) and np.linalg.norm(blk) < tau * ref[k]:
                a[sl[k], sl[j]] = 0.0
                a[sl[j], sl[k]] = 0.0
        u_rows[k] = {j: a[sl[k], sl[j]].copy() for j in [k] + later}
        dk = a[sl[k], sl[k]]
        for i in later:
            zi = np.linalg.solve(dk, a[sl[k], sl[i]])
            for j in later:
                a[sl[i], sl[j]] -= zi.T @ a[sl[k], sl[j]]

    def solve(r):
        z = r.astype(float).copy()
        for k in order:
            dz = np.linalg.solve(u_rows[k][k], z[sl[k]])
            for j, ukj in u_rows[k].items():
                if j != k:
                    z[sl[j]] -= ukj.T @ dz
        x = np.zeros_like(z)
        for i in reversed(order):
            acc = z[sl[i]].copy()
            for j, uij in u_rows[i].items():
                if j != i:
                    acc -= uij @ x[sl[j]]
            x[sl[i]] = np.linalg.solve(u_rows[i][i], acc)
        return x
    return solve


def test_sym_ilut_ends_are_ilu0_and_exact(ifmm_case):
    """The symmetric threshold factorisation: tau = infinity is block ILU(0),
    tau = 0 keeps the whole structural fill (half of it above the diagonal)
    and solves S exactly."""
    x, fine, coarse, sp, order = ifmm_case[1e-2]
    r = np.random.default_rng(11).standard_normal((sp.n, 2))
    il = oracle.SymBlockILUT(sp, np.inf, order)
    assert il.kept_fill == 0 and il.dropped > 0
    want = oracle.BlockILU0(sp, order).solve(r)
    assert np.abs(il.solve(r) - want).max() <= 1e-12 * np.abs(want).max()
    ex = oracle.SymBlockILUT(sp, 0.0, order)
    assert ex.dropped == 0
    assert 2 * ex.kept_fill == len(oracle.block_fill(sp, order)) - len(sp.s_blocks)
    want = np.linalg.solve(oracle.dense_s(sp), r)
    assert np.abs(ex.solve(r) - want).max() <= 1e-11 * np.abs(want).max()


@pytest.mark.parametrize("tau", [1e-4, 3e-5, 1e-5])
def test_sym_ilut_against_dense_brute_force(ifmm_case, tau):
    """Against a right-looking factorisation of the dense S with the same drop
    rule (different order of the updates), and the preconditioner it gives
    is a symmetric operator.  The tolerances keep part of the fill and drop
    the rest (43, 80 and 193 of 1028 fill blocks kept at N = 1500)."""
    x, fine, coarse, sp, order = ifmm_case[1e-2]
    il = oracle.SymBlockILUT(sp, tau, order)
    assert il.dropped > 0 and il.kept_fill > 0
    brute = _dense_sym_ilut(sp, tau, order)
    r = np.random.default_rng(12).standard_normal((sp.n, 3))
    got, want = il.solve(r), brute(r)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()
    assert abs(r[:, 1] @ got[:, 0] - r[:, 0] @ got[:, 1]) <= 1e-11 * np.abs(r[:, 0] @ got[:, 0])


def test_sym_ilut_fill_shrinks_with_tau(ifmm_case):
    x, fine, coarse, sp, order = ifmm_case[1e-2]
    kept = [oracle.SymBlockILUT(sp, t, order).kept_fill for t in (0.0, 1e-3, 1e-2, 1e-1)]
    assert all(a >= b for a, b in zip(kept, kept[1:])) and kept[0] > kept[-1]


@pytest.mark.parametrize("d", [1e-3, 1e-2])
def test_gmres_with_sym_ilut_preconditioner(ifmm_case, d):
    """Section 5.5's setup with the symmetric threshold factorisation."""
    x, fine, coarse, sp, order = ifmm_case[d]
    il = oracle.SymBlockILUT(sp, 1e-2, order)
    pre = lambda v: oracle.apply_v(sp, il.solve(oracle.apply_ut(sp, v)))
    b = np.random.default_rng(13).standard_normal((fine.tree.n, 2))
    xs, hist = oracle.gmres(fine.matvec, b, pre, tol=1e-10)
    assert max(len(h) for h in hist) <= 20
    want = np.linalg.solve(fine.dense(), b)
    assert np.abs(xs - want).max() <= 1e-7 * np.abs(want).max()
