"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own formulas: LAPACK QR,
dense linear algebra, brute force over index pairs, closed forms of special
cases and the identities the paper states (orthogonality of U and V, S of the
size of A, A = U S V^T exactly, symmetry / positive definiteness of S).
"""

import importlib
import os

import numpy as np
import pytest
import scipy.linalg as sla

import h2inputs
import oracle
from oracle import h2 as oh2
from oracle import householder as ohh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _h2(kind, n, seed, leaf, cheb, tol=0.0, cap=0, eta=1.0, kernel=None, scale=None):
    x = h2inputs.points(kind, n, seed)
    if scale is None:
        scale = 1.0 / n if x.shape[1] == 2 else 1.0 / (4 * np.pi * n)
    return oracle.build_h2(x, leaf, cheb, scale, 1.0, tol, cap, eta, kernel)


CASES = [
    ("square", 1024, 1, 32, 4, 0.0, 16),      # the 2D Chebyshev 4x4 workload, fixed rank 16
    ("cube", 1536, 11, 32, 3, 1e-8, 27),      # 3D, recompressed, uneven ranks
    ("sphere", 2048, 12, 64, 3, 1e-8, 27),    # 2-manifold, recompressed
    ("torus", 777, 13, 24, 3, 1e-8, 20),      # ragged sizes, rank cap below 27
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def case(request):
    kind, n, seed, leaf, cheb, tol, cap = request.param
    h2 = _h2(kind, n, seed, leaf, cheb, tol, cap)
    sp = oracle.sparsify(h2)
    a = h2.dense()
    u = oracle.dense_u(sp)
    s = oracle.dense_s(sp)
    return h2, sp, a, u, s


# ----------------------------------------------------------------- inputs

def test_splitmix_golden():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        want = [int(line, 16) for line in f if line.strip() and not line.startswith("#")]
    got = [int(v) for v in h2inputs.splitmix64(0, 3)]
    assert got == want


def test_points_in_domain():
    assert np.all((h2inputs.points_cube(1000, 3) >= 0) & (h2inputs.points_cube(1000, 3) < 1))
    sph = h2inputs.points_sphere(1000, 2)
    assert np.allclose((sph * sph).sum(1), 1.0, atol=1e-14)
    tor = h2inputs.points_torus(1000, 4)
    ring = np.sqrt(tor[:, 0] ** 2 + tor[:, 1] ** 2) - 1.0
    assert np.allclose(ring ** 2 + tor[:, 2] ** 2, 0.35 ** 2, atol=1e-12)


# ----------------------------------------------------------------- Householder

@pytest.mark.parametrize("shape", [(32, 16), (20, 27), (64, 64), (54, 27), (7, 1), (1, 5)])
def test_householder_matches_lapack(shape):
    rng = np.random.default_rng(sum(shape))
    b = rng.standard_normal(shape)
    q, r = ohh.householder_qr(b)
    q_ref, r_ref = sla.qr(b, mode="full")
    assert np.abs(q - q_ref).max() < 1e-13
    assert np.abs(r - r_ref).max() < 1e-13 * max(1.0, np.abs(r_ref).max())
    assert np.abs(q.T @ q - np.eye(shape[0])).max() < 1e-14


def test_householder_zero_subcolumn():
    b = np.array([[2.0, 1.0], [0.0, 3.0], [0.0, 4.0]])
    q, r = ohh.householder_qr(b)
    q_ref, r_ref = sla.qr(b, mode="full")
    assert np.abs(q - q_ref).max() < 1e-15 and np.abs(r - r_ref).max() < 1e-14
    assert r[0, 0] == 2.0  # tau = 0: the first reflector is the identity


# ----------------------------------------------------------------- trees

@pytest.mark.parametrize("kind,n,leaf", [("square", 300, 8), ("cube", 500, 16), ("torus", 257, 5)])
def test_cluster_tree_rules(kind, n, leaf):
    x = h2inputs.points(kind, n, 5)
    tr = oracle.build_cluster_tree(x, leaf)
    assert sorted(tr.perm.tolist()) == list(range(n))
    leaves = tr.clusters_at_level(0)
    assert tr.size[leaves].max() <= leaf
    assert tr.depth == 0 or tr.size[leaves].max() * 2 > leaf or (n + (1 << tr.depth) - 1) >> (tr.depth - 1) > leaf
    assert set(tr.size[leaves].tolist()) <= {n >> tr.depth, (n + (1 << tr.depth) - 1) >> tr.depth}
    for c in range(tr.ncl):
        pts = x[tr.perm[tr.start[c]:tr.start[c] + tr.size[c]]]
        assert np.array_equal(pts.min(0), tr.lo[c]) and np.array_equal(pts.max(0), tr.hi[c])
        if 2 * c + 1 < tr.ncl:
            axis = int(np.argmax(tr.hi[c] - tr.lo[c]))
            left = x[tr.perm[tr.start[2 * c + 1]:tr.start[2 * c + 1] + tr.size[2 * c + 1]], axis]
            right = x[tr.perm[tr.start[2 * c + 2]:tr.start[2 * c + 2] + tr.size[2 * c + 2]], axis]
            assert left.max() <= right.min()
            assert tr.size[2 * c + 1] == tr.size[c] // 2


@pytest.mark.parametrize("kind,n,leaf,eta", [("square", 400, 8, 1.0), ("cube", 600, 12, 1.0),
                                             ("cube", 300, 8, 0.0)])
def test_block_tree_partition_and_monotone(kind, n, leaf, eta):
    x = h2inputs.points(kind, n, 6)
    tr = oracle.build_cluster_tree(x, leaf)
    bt = oracle.build_block_tree(tr, eta)
    cover = np.zeros((n, n), dtype=np.int64)

    def rows(c):
        return slice(tr.start[c], tr.start[c] + tr.size[c])

    for t, s in bt.near[0]:
        cover[rows(t), rows(s)] += 1
    for k in range(tr.depth + 1):
        for t, s in bt.far[k]:
            cover[rows(t), rows(s)] += 1
            if eta > 0:
                # admissibility on boxes bounds the point distances from below
                pt = x[tr.perm[rows(t)]]
                ps = x[tr.perm[rows(s)]]
                dmin = np.sqrt(((pt[:, None] - ps[None]) ** 2).sum(-1)).min()
                diam = max(np.sqrt(((tr.hi[t] - tr.lo[t]) ** 2).sum()),
                           np.sqrt(((tr.hi[s] - tr.lo[s]) ** 2).sum()))
                assert dmin >= diam * (1 - 1e-12)
            if k > 0:
                kids_t = np.array([2 * t + 1, 2 * t + 1, 2 * t + 2, 2 * t + 2])
                kids_s = np.array([2 * s + 1, 2 * s + 2, 2 * s + 1, 2 * s + 2])
                assert oracle.admissible(tr, kids_t, kids_s, eta).all()
    assert (cover == 1).all()


# ----------------------------------------------------------------- H^2 construction

def test_chebyshev_nestedness():
    h2 = _h2("cube", 1200, 7, 32, 3)
    tr = h2.tree
    for c in range(1, tr.ncl):
        p = (c - 1) // 2
        if not h2.ff[p] or 2 * c + 1 >= tr.ncl:
            continue
        # father's basis restricted to the son's points equals the son's basis times T
        st = tr.start[c]
        pts = h2.x_tree[st:st + tr.size[c]]
        father_on_son = oh2.tensor_lagrange(*oh2.padded_box(tr.lo[p], tr.hi[p]), 3, pts)
        son = oh2.tensor_lagrange(*oh2.padded_box(tr.lo[c], tr.hi[c]), 3, pts)
        np.testing.assert_allclose(son @ h2.transfer[c], father_on_son, atol=1e-12)


def test_matvec_matches_dense(case):
    h2, sp, a, u, s = case
    v = np.random.default_rng(0).standard_normal((h2.tree.n, 3))
    assert np.abs(h2.matvec(v) - a @ v).max() <= 1e-13 * np.abs(a @ v).max()


def _invdist_exact(h2):
    """c / |x_i - x_j| off the diagonal and A_ii = diag, from scipy's pairwise
    distances (independent of the oracle's kernel code)."""
    from scipy.spatial.distance import cdist
    d = cdist(h2.x_tree, h2.x_tree)
    np.fill_diagonal(d, 1.0)
    exact = h2.scale / d
    np.fill_diagonal(exact, h2.diag)
    return exact


def test_h2_close_to_kernel(case):
    h2, sp, a, u, s = case
    exact = _invdist_exact(h2)
    assert np.linalg.norm(a - exact) <= 1e-4 * np.linalg.norm(exact)
    # the diagonal is the prescribed value exactly (it lies in the close part)
    assert np.array_equal(np.diag(a), np.full(h2.tree.n, h2.diag))


# ------------------------------------------------ inverse distance c / |x - y|

def test_invdist_kernel_values_by_hand():
    """Entries of c / |x_i - x_j| with A_ii = 1 (the benchmark matrices) for
    four points at distances 1/2, 1, 3/2, sqrt 2 and sqrt 3, written out by
    hand, for the close blocks and the kernel blocks of the far field."""
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 1.0], [0.5, 0.0, 0.0]])
    idx = np.arange(4)
    c = 0.25
    r2, r3 = 0.17677669529663688, 0.14433756729740643   # c / sqrt 2, c / sqrt 3
    want = np.array([[1.0, 0.25, r2, 0.5],
                     [0.25, 1.0, r3, 0.5],
                     [r2, r3, 1.0, 0.25 / 1.5],
                     [0.5, 0.5, 0.25 / 1.5, 1.0]])
    got = oh2.close_block(x, idx, idx, c, 1.0)
    assert np.abs(got - want).max() <= 2e-16
    # a close block between different index sets has no diagonal rule
    got = oh2.close_block(x, np.array([0, 3]), np.array([1, 2]), c, 1.0)
    assert np.abs(got - want[np.ix_([0, 3], [1, 2])]).max() <= 2e-16
    far = oh2.kernel_block(x[:2], x[2:], c)
    assert np.abs(far - want[:2, 2:]).max() <= 2e-16


@pytest.mark.parametrize("kind,n,seed,leaf", [("cube", 1536, 11, 32), ("square", 1024, 1, 32)])
def test_invdist_h2_approximates_pairwise_distances(kind, n, seed, leaf):
    """The Chebyshev H^2 of c / |x - y| against the dense matrix from scipy's
    pairwise distances: the off-diagonal error is small and falls at least
    fivefold from Chebyshev order 3 to 4 (interpolation of a smooth far
    field), so a wrong power, sign or term in the far field fails."""
    err = {}
    for cheb in (3, 4):
        h2 = _h2(kind, n, seed, leaf, cheb)
        exact = _invdist_exact(h2)
        off = ~np.eye(n, dtype=bool)
        err[cheb] = np.linalg.norm((h2.dense() - exact)[off]) / np.linalg.norm(exact[off])
    assert err[3] <= 1e-3
    assert err[4] <= err[3] / 5


def test_invdist_pins_catch_a_squared_distance(monkeypatch):
    """c / |r|^2 in place of c / |r| (in the far field, then in the close
    field) is caught by the comparison with scipy's pairwise distances."""
    good_k, good_c = oh2.kernel_block, oh2.close_block

    def bad_kernel(xr, xc, scale, kernel=None):
        if kernel is None:
            d = xr[:, None, :] - xc[None, :, :]
            return scale / (d * d).sum(axis=2)
        return good_k(xr, xc, scale, kernel)

    def bad_close(x, ti, si, scale, diag, kernel=None):
        out = good_c(x, ti, si, scale, diag, kernel)
        if kernel is None:
            same = ti[:, None] == si[None, :]
            out = np.where(same, diag, out * out / scale)
        return out

    for name, fn in (("kernel_block", bad_kernel), ("close_block", bad_close)):
        with monkeypatch.context() as m:
            m.setattr(oh2, name, fn)
            h2 = _h2("cube", 1536, 11, 32, 3)
            exact = _invdist_exact(h2)
            assert np.linalg.norm(h2.dense() - exact) > 1e-2 * np.linalg.norm(exact - np.eye(1536)), name


def test_recompressed_bases_orthonormal():
    h2 = _h2("sphere", 2048, 12, 64, 3, 1e-8, 27)
    ranks = h2.rank[h2.ff]
    assert ranks.max() <= 27 and len(np.unique(ranks)) > 1
    for t, b in h2.leaf_basis.items():
        assert np.abs(b.T @ b - np.eye(b.shape[1])).max() < 1e-13
    for t in range(h2.tree.ncl):
        if h2.ff[t] and 2 * t + 1 < h2.tree.ncl and (2 * t + 1) in h2.transfer:
            st = np.vstack([h2.transfer[2 * t + 1], h2.transfer[2 * t + 2]])
            assert np.abs(st.T @ st - np.eye(st.shape[1])).max() < 1e-13
    # truncation at 1e-8 keeps the Chebyshev H^2 matrix
    cheb = _h2("sphere", 2048, 12, 64, 3)
    assert np.linalg.norm(h2.dense() - cheb.dense()) <= 1e-7 * np.linalg.norm(cheb.dense())


# ----------------------------------------------------------------- the factorisation

def test_sizes(case):
    h2, sp, a, u, s = case
    assert sp.nonbasis.sum() == h2.tree.n          # S is N x N (eq. usv)
    assert s.shape == a.shape
    assert (sp.kept <= sp.n_act).all() and (sp.kept[0] == 0)


def test_u_orthogonal(case):
    h2, sp, a, u, s = case
    assert np.abs(u.T @ u - np.eye(u.shape[0])).max() <= 1e-13
    for t, q in sp.q.items():
        assert np.abs(q.T @ q - np.eye(q.shape[0])).max() <= 1e-13


def test_exact_reconstruction(case):
    h2, sp, a, u, s = case
    assert np.linalg.norm(u @ s @ u.T - a) <= 1e-12 * np.linalg.norm(a)


def test_structural_zeros_and_pattern(case):
    h2, sp, a, u, s = case
    full = u.T @ a @ u                                   # brute-force S
    mask = np.zeros(full.shape, dtype=bool)
    for (t, v) in sp.s_blocks:
        mask[sp.soff[t]:sp.soff[t] + sp.nonbasis[t], sp.soff[v]:sp.soff[v] + sp.nonbasis[v]] = True
    assert np.abs(full[~mask]).max() <= 1e-14 * np.abs(a).max()
    assert np.abs(full[mask] - s[mask]).max() <= 1e-13 * np.abs(a).max()
    assert oracle.pattern_predicate(sp) == set(sp.s_blocks)


def test_symmetry_and_spectrum(case):
    h2, sp, a, u, s = case
    assert np.abs(s - s.T).max() <= 1e-13 * np.abs(s).max()
    ev_s = np.linalg.eigvalsh(0.5 * (s + s.T))
    ev_a = np.linalg.eigvalsh(0.5 * (a + a.T))
    assert np.abs(ev_s - ev_a).max() <= 1e-12 * np.abs(ev_a).max()
    # Proposition 2.1: A SPD => S SPD (the 2D workload with c = 1/N is indefinite:
    # nearly coincident points give off-diagonal entries above the unit diagonal)
    assert (ev_s.min() > 0) == (ev_a.min() > 0)


def test_polynomial_kernel_exact():
    """(1 + x.y)^2 has degree 2 per axis: Chebyshev order 3 reproduces it exactly."""
    def kern(xr, xc):
        return (1.0 + (xr * xc).sum(-1)) ** 2
    h2 = _h2("cube", 700, 9, 16, 3, kernel=kern)
    sp = oracle.sparsify(h2)
    k_dense = kern(h2.x_tree[:, None, :], h2.x_tree[None, :, :])
    u, s = oracle.dense_u(sp), oracle.dense_s(sp)
    assert np.linalg.norm(h2.dense() - k_dense) <= 1e-12 * np.linalg.norm(k_dense)
    assert np.linalg.norm(u @ s @ u.T - k_dense) <= 1e-12 * np.linalg.norm(k_dense)


def test_single_leaf_is_identity():
    h2 = _h2("square", 30, 3, 32, 4)
    sp = oracle.sparsify(h2)
    assert h2.tree.depth == 0 and sp.kept[0] == 0
    assert np.array_equal(sp.q[0], np.eye(30))
    assert np.array_equal(oracle.dense_s(sp), h2.dense())


def test_weak_admissibility_closed_form():
    """HODLR special case: pattern = own block + strips to ancestors; ILU(0) exact."""
    h2 = _h2("square", 512, 8, 16, 4, eta=0.0)
    sp = oracle.sparsify(h2)
    tr = h2.tree
    want = set()
    for t in range(tr.ncl):
        if sp.nonbasis[t] == 0:
            continue
        c = t
        while True:
            if sp.nonbasis[c] > 0:
                want.add((t, c))
                want.add((c, t))
            if c == 0 or sp.kept[c] == 0:
                break
            c = (c - 1) // 2
    assert set(sp.s_blocks) == want
    b = np.random.default_rng(1).standard_normal((tr.n, 2))
    ilu = oracle.BlockILU0(sp)
    exact = np.linalg.solve(oracle.dense_s(sp), b)
    assert np.abs(ilu.solve(b) - exact).max() <= 1e-12 * np.abs(exact).max()


def test_solve_dense_lu(case):
    h2, sp, a, u, s = case
    b = np.random.default_rng(2).standard_normal((h2.tree.n, 2))
    x = oracle.apply_v(sp, oracle.dense_lu_solver(sp)(oracle.apply_ut(sp, b)))
    ref = np.linalg.solve(a, b)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


def test_ilu0_full_pattern_is_lu():
    """Two near leaves only: every block of S is present, so ILU(0) is the LU."""
    h2 = _h2("square", 60, 4, 32, 4)
    sp = oracle.sparsify(h2)
    assert h2.tree.depth == 1 and not h2.bt.far[0].size
    b = np.random.default_rng(3).standard_normal((60, 1))
    ref = np.linalg.solve(oracle.dense_s(sp), b)
    assert np.abs(oracle.BlockILU0(sp).solve(b) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_refinement_with_ilu0(case):
    h2, sp, a, u, s = case
    b = np.random.default_rng(4).standard_normal((h2.tree.n, 2))
    x, hist = oracle.refine(sp, oracle.BlockILU0(sp).solve, b, 1e-12)
    assert hist[-1] <= 1e-12 and len(hist) <= 10
    ref = np.linalg.solve(a, b)
    assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()


def test_elimination_order_colouring(case):
    """Greedy colouring: valid (no block of S joins one colour on one level) and minimal."""
    h2, sp, a, u, s = case
    tr = h2.tree
    col = oracle.elimination_colours(sp)
    order = oracle.elimination_order(sp)
    assert sorted(order) == sorted(c for c in range(tr.ncl) if sp.nonbasis[c] > 0)
    keys = [(tr.level(c), col[c], c) for c in order]
    assert keys == sorted(keys)
    nbrs = {}
    for (t, v) in sp.s_blocks:
        if t != v and tr.level(t) == tr.level(v):
            assert col[t] != col[v]
            nbrs.setdefault(t, set()).add(v)
    for t, c in col.items():
        earlier = {col[v] for v in nbrs.get(t, ()) if v < t}
        assert all(k in earlier for k in range(c))        # smallest free colour
    b = np.random.default_rng(9).standard_normal((tr.n, 1))
    x, hist = oracle.refine(sp, oracle.BlockILU0(sp, order).solve, b, 1e-12)
    ref = np.linalg.solve(a, b)
    assert hist[-1] <= 1e-12 and np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()


def test_ilu0_full_pattern_is_lu_in_any_order():
    h2 = _h2("square", 60, 4, 32, 4)
    sp = oracle.sparsify(h2)
    b = np.random.default_rng(3).standard_normal((60, 1))
    ref = np.linalg.solve(oracle.dense_s(sp), b)
    for order in (list(sp.order)[::-1], oracle.elimination_order(sp)):
        assert np.abs(oracle.BlockILU0(sp, order).solve(b) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_block_fill_gives_exact_factor(case):
    """Block ILU(0) on the pattern closed under graph elimination is the exact
    block factorisation: it reproduces the dense solve of S (Sections 5.3-5.4
    use a sparse direct factorisation).  The fill is idempotent and the
    unfilled ILU(0) is not exact, so the pin tells the two apart."""
    h2, sp, a, u, s = case
    order = oracle.elimination_order(sp)
    fill = oracle.block_fill(sp, order)
    assert set(sp.s_blocks) <= fill
    assert oracle.block_fill(oracle.filled(sp, order), order) == fill
    b = np.random.default_rng(6).standard_normal((h2.tree.n, 2))
    ref = np.linalg.solve(s, b)
    got = oracle.BlockILU0(oracle.filled(sp, order), order).solve(b)
    err = np.abs(got - ref).max()
    assert err <= 1e-11 * np.abs(ref).max()
    if len(fill) > len(sp.s_blocks):
        ilu = oracle.BlockILU0(sp, order).solve(b)
        assert np.abs(ilu - ref).max() > 100 * max(err, 1e-15 * np.abs(ref).max())


def test_block_fill_brute_force():
    """Tiny pattern: fill against elimination of a dense boolean matrix."""
    h2 = _h2("square", 400, 8, 16, 3)
    sp = oracle.sparsify(h2)
    order = oracle.elimination_order(sp)
    fill = oracle.block_fill(sp, order)
    idx = {c: i for i, c in enumerate(order)}
    n = len(order)
    g = np.zeros((n, n), dtype=bool)
    for (t, v) in sp.s_blocks:
        g[idx[t], idx[v]] = True
    for k in range(n):                      # symbolic Gaussian elimination
        later = [j for j in range(k + 1, n) if g[k, j]]
        for i in later:
            for j in later:
                g[i, j] = True
    want = {(order[i], order[j]) for i in range(n) for j in range(n) if g[i, j]}
    assert fill == want


def test_cg_reference(case):
    h2, sp, a, u, s = case
    b = np.random.default_rng(5).standard_normal((h2.tree.n, 1))
    x = oracle.conjugate_gradient(h2.matvec, b, tol=1e-14)
    ref = np.linalg.solve(a, b)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


# ----------------------------------------------------------------- planted mistakes

def test_pins_catch_a_dropped_reflector(monkeypatch):
    """A Q missing its last reflector breaks orthogonal completion: pins fail."""
    good = ohh.householder_qr

    def bad(b):
        q, r = good(b)
        q = q.copy()
        q[:, -1] *= -1.0       # still orthogonal, but Q^T B no longer has zero rows
        q[:, 0], q[:, -1] = q[:, -1].copy(), q[:, 0].copy()
        return q, q.T @ b

    monkeypatch.setattr(importlib.import_module("oracle.sparsify"), "householder_qr", bad)
    h2 = _h2("square", 256, 3, 16, 4)
    sp = oracle.sparsify(h2)
    a, u, s = h2.dense(), oracle.dense_u(sp), oracle.dense_s(sp)
    assert np.linalg.norm(u @ s @ u.T - a) > 1e-6 * np.linalg.norm(a)


def test_pins_catch_a_transposed_coupling(monkeypatch):
    """Using D_ts^T for the coupling changes A_H2 relative to the dense build."""
    h2 = _h2("cube", 600, 3, 16, 3)
    a_ref = h2.dense()
    orig = oh2.H2Matrix.coupling
    monkeypatch.setattr(oh2.H2Matrix, "coupling", lambda self, t, s: orig(self, t, s).T)
    sp = oracle.sparsify(h2)
    u, s = oracle.dense_u(sp), oracle.dense_s(sp)
    assert np.linalg.norm(u @ s @ u.T - a_ref) > 1e-10 * np.linalg.norm(a_ref)


# ------------------------------------------------ Example 5.2: exp(-|r|^2) core

def test_exp_kernel_values_by_hand():
    """Entries of 2 delta_ij + exp(-|r_i - r_j|^2) (Example 5.2) for three
    points at squared distances 1, 2 and 3, written out by hand."""
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 1.0]])
    idx = np.arange(3)
    got = oh2.close_block(x, idx, idx, 1.0, 3.0, oracle.EXP)
    e1, e2, e3 = 0.36787944117144233, 0.1353352832366127, 0.049787068367863944
    want = np.array([[3.0, e1, e2], [e1, 3.0, e3], [e2, e3, 3.0]])
    assert np.abs(got - want).max() <= 2e-16 * 3
    far = oh2.kernel_block(x[:1], x[1:], 0.5, oracle.EXP)
    assert np.abs(far - 0.5 * np.array([[e1, e2]])).max() <= 1e-17


@pytest.fixture(scope="module")
def exp_case():
    x = h2inputs.points("cube", 1536, 11)
    out = {}
    for cheb in (3, 4):
        out[cheb] = oracle.build_h2(x, 32, cheb, 1.0, 3.0, 1e-8, 64, 1.0, oracle.EXP)
    return out


def test_exp_h2_approximates_the_kernel(exp_case):
    """The Chebyshev H^2 of the exp core against the dense matrix from
    scipy's pairwise distances: small, and shrinking with the order."""
    from scipy.spatial.distance import cdist
    err = {}
    for cheb, h2 in exp_case.items():
        exact = np.exp(-cdist(h2.x_tree, h2.x_tree, "sqeuclidean")) + 2.0 * np.eye(h2.tree.n)
        err[cheb] = np.linalg.norm(h2.dense() - exact) / np.linalg.norm(exact)
    assert err[4] <= 1e-4
    assert err[4] <= err[3] / 5


def test_exp_sparsification_is_exact_and_spd(exp_case):
    """A = U S U^T to rounding for the exp core too; S inherits the
    positive definiteness of 2 I + (a Gaussian Gram matrix)."""
    h2 = exp_case[4]
    sp = oracle.sparsify(h2)
    a = h2.dense()
    u = oracle.dense_u(sp)
    s = oracle.dense_s(sp)
    assert np.linalg.norm(u @ s @ u.T - a) <= 1e-12 * np.linalg.norm(a)
    assert np.abs(u.T @ u - np.eye(u.shape[0])).max() <= 1e-13
    assert np.linalg.eigvalsh(0.5 * (s + s.T)).min() > 1.9


def test_exp_pins_catch_a_dropped_square(monkeypatch):
    """A far field of exp(-|r|) instead of exp(-|r|^2) (the close field kept
    right) is caught by the comparison with scipy's pairwise distances."""
    from scipy.spatial.distance import cdist
    good = oh2.kernel_block

    def bad(xr, xc, scale, kernel=None):
        if kernel == oracle.EXP:
            d = xr[:, None, :] - xc[None, :, :]
            return scale * np.exp(-np.sqrt((d * d).sum(axis=2)))
        return good(xr, xc, scale, kernel)

    monkeypatch.setattr(oh2, "kernel_block", bad)
    x = h2inputs.points("cube", 1536, 11)
    h2 = oracle.build_h2(x, 32, 4, 1.0, 3.0, 1e-8, 64, 1.0, oracle.EXP)
    exact = np.exp(-cdist(h2.x_tree, h2.x_tree, "sqeuclidean")) + 2.0 * np.eye(h2.tree.n)
    assert np.linalg.norm(h2.dense() - exact) > 1e-2 * np.linalg.norm(exact)


def test_s_rows_stay_sparse_as_depth_grows():
    """Section 3 and the nnz study of Section 5.1: S stays sparse.  In a leaf
    row, the blocks whose column cluster sits k levels up fall off
    geometrically with k, so a row's block count is bounded whatever the
    depth (at these N the total still rises towards that bound)."""
    import collections
    n = 8192
    x = h2inputs.points("square", n, 3)
    h2 = oracle.build_h2(x, 32, 4, 1.0 / n, 1.0, 1e-6, 0, 1.0)
    sp = oracle.sparsify(h2)
    tr = h2.tree
    assert tr.depth >= 7
    leaves = [c for c in range(tr.ncl) if 2 * c + 1 >= tr.ncl and sp.nonbasis[c] > 0]
    per_level = collections.Counter()
    for (t, s) in sp.s_blocks:
        if 2 * t + 1 >= tr.ncl:
            per_level[tr.level(s)] += 1
    counts = [per_level[lv] / len(leaves) for lv in sorted(per_level)]
    assert len(counts) >= 5
    for a, b in zip(counts[1:], counts[2:]):
        assert b <= 0.75 * a
    assert sum(counts) <= 4 * counts[0] + counts[1]


def test_nonsymmetric_kernel_over_a_shared_basis():
    """Section 2 derives A = U S V^T without symmetry.  With a non-symmetric
    kernel over one Chebyshev basis per cluster (U = V, no recompression),
    the sweep still reproduces A_H2 exactly, S comes out non-symmetric, and
    the exact block factorisation of S solves A_H2 x = b like a dense LU."""
    from scipy.spatial.distance import cdist

    def kern(a, b):
        d = a - b
        return (1.0 + 0.5 * d[..., 0]) / np.sqrt((d * d).sum(axis=-1) + 1e-4)

    n = 1200
    x = h2inputs.points("cube", n, 31)
    h2 = oracle.build_h2(x, 32, 4, 1.0, 1.0, 0.0, 0, 1.0, kern)
    a = h2.dense()
    xt = h2.x_tree
    exact = (1.0 + 0.5 * (xt[:, None, 0] - xt[None, :, 0])) / np.sqrt(cdist(xt, xt, "sqeuclidean") + 1e-4)
    assert np.linalg.norm(a - exact) <= 1e-4 * np.linalg.norm(exact)
    assert np.abs(a - a.T).max() > 1e-3 * np.abs(a).max()
    sp = oracle.sparsify(h2)
    u, s = oracle.dense_u(sp), oracle.dense_s(sp)
    assert np.linalg.norm(u @ s @ u.T - a) <= 1e-12 * np.linalg.norm(a)
    assert np.abs(s - s.T).max() > 1e-3 * np.abs(s).max()
    order = oracle.elimination_order(sp)
    lu = oracle.BlockILU0(oracle.filled(sp, order), order)
    b = np.random.default_rng(1).standard_normal((n, 2))
    got = oracle.apply_v(sp, lu.solve(oracle.apply_ut(sp, b)))
    want = np.linalg.solve(a, b)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()
