"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Inputs are seeded and synthetic; every case spans several tiles and ragged
cluster sizes.  Bars:
  * permutation, ranks, sizes, S offsets and the S block pattern: bit-exact;
  * FP64 path: Q_t and S blocks within 1e-12 of the oracle (relative to the
    largest entry of A), H^2 matvec within 1e-13;
  * mixed path (FP32 transforms on MFMA): S blocks within 5e-6;
  * solves: relative residual <= the requested tolerance, and x within
    1e-8 of the dense solve of A_H2.
The oracle's H^2 coefficients are handed to the library through h2_import so
that both sides sparsify the same H^2 matrix (the recompressed bases are only
defined up to a rotation inside each kept subspace); the library's own
construction is compared through basis-independent quantities.
"""

import sys

import numpy as np
import pytest

import oracle
import paper_1705_04601_amd as P
from h2test_util import import_arrays, make_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "square1k": ("square", 1024, 1, 32, 4, 0.0, 16, 1.0),    # the 2D fixed-rank workload itself
    "cube1536": ("cube", 1536, 11, 32, 3, 1e-8, 27, 1.0),
    "sphere2k": ("sphere", 2048, 12, 64, 3, 1e-8, 27, 1.0),
    "torus777": ("torus", 777, 13, 24, 3, 1e-8, 20, 1.0),
    "cube2500r48": ("cube", 2500, 8, 40, 4, 1e-8, 48, 1.0),
    "hodlr700": ("square", 700, 9, 16, 4, 0.0, 16, 0.0),
}
_cache = {}


def case(name):
    if name not in _cache:
        kind, n, seed, leaf, cheb, tol, cap, eta = CASES[name]
        x, sc, h2 = make_case(kind, n, seed, leaf, cheb, tol, cap, eta)
        sp = oracle.sparsify(h2)
        a = h2.dense()
        _cache[name] = (x, sc, h2, sp, a, (leaf, cheb, tol, cap, eta))
    return _cache[name]


def note(msg):
    sys.stderr.write(f"[gpu-case] {msg}\n")
    sys.stderr.flush()


def dev(arr):
    """(n, nrhs) float64 column-major CUDA tensor."""
    arr = np.asarray(arr, dtype=np.float64)
    if arr.ndim == 1:
        arr = arr[:, None]
    return torch.from_numpy(np.ascontiguousarray(arr.T)).cuda().T


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def imported(name):
    x, sc, h2, sp, a, (leaf, cheb, tol, cap, eta) = case(name)
    return P.h2_import(x, sc, 1.0, leaf, cheb, eta, *import_arrays(h2))


def to_tree(v, perm):
    return v[perm]


def from_tree(v_tree, perm):
    out = np.empty_like(v_tree)
    out[perm] = v_tree
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_imported(name):
    x, sc, h2, sp, a, _ = case(name)
    note(f"matvec imported {name}")
    h = imported(name)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((x.shape[0], 3))
    y = dev(np.zeros_like(v))
    P.h2_matvec(h, dev(v), y)
    want = from_tree(a @ to_tree(v, h2.tree.perm), h2.tree.perm)
    assert np.abs(host(y) - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_own_build(name):
    x, sc, h2, sp, a, (leaf, cheb, tol, cap, eta) = case(name)
    note(f"matvec own build {name}")
    h = P.h2_build(x, sc, 1.0, leaf, cheb, tol, cap, eta)
    v = np.random.default_rng(2).standard_normal((x.shape[0], 2))
    y = dev(np.zeros_like(v))
    P.h2_matvec(h, dev(v), y)
    want = from_tree(a @ to_tree(v, h2.tree.perm), h2.tree.perm)
    assert np.abs(host(y) - want).max() <= 1e-10 * np.abs(want).max()


@pytest.mark.parametrize("name", ["cube1536", "sphere2k", "torus777"])
def test_matvec_close_generated_vs_resident(name, monkeypatch):
    """The close part from kernel blocks written out once (the default) and
    generated inside the GEMM for every product: both against the dense
    product, and against each other (the same values in the same order)."""
    x, sc, h2, sp, a, _ = case(name)
    note(f"matvec close resident vs generated {name}")
    v = np.random.default_rng(3).standard_normal((x.shape[0], 5))
    want = from_tree(a @ to_tree(v, h2.tree.perm), h2.tree.perm)
    got = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("H2SP_CLOSE_RESIDENT", flag)
        h = imported(name)  # a fresh handle: the plan (and the choice) is per matrix
        y = dev(np.zeros_like(v))
        P.h2_matvec(h, dev(v), y)
        got[flag] = host(y)
        assert np.abs(got[flag] - want).max() <= 1e-13 * np.abs(want).max()
    assert np.abs(got["0"] - got["1"]).max() <= 1e-15 * np.abs(want).max()


def _check_plan(sph, sp):
    """Sizes, S offsets, elimination order and the stored pattern: bit-exact."""
    plan = P.h2_sparse_export_plan(sph)
    assert np.array_equal(plan["n_act"], sp.n_act)
    assert np.array_equal(plan["kept"], sp.kept)
    assert np.array_equal(plan["nonbasis"], sp.nonbasis)
    assert np.array_equal(plan["soff"], sp.soff)
    elim = [int(c) for c in plan["elim"] if sp.nonbasis[c] > 0]
    assert elim == oracle.elimination_order(sp)
    pos = {int(c): i for i, c in enumerate(plan["elim"])}
    got = set()
    for i, t in enumerate(plan["elim"]):
        for b in range(plan["rowptr"][i], plan["rowptr"][i + 1]):
            got.add((int(t), int(plan["colidx"][b])))
    want = {(t, s) for (t, s) in sp.s_blocks if pos[t] <= pos[s]}
    assert got == want
    return plan


@pytest.mark.parametrize("name", list(CASES))
def test_sparsify_fp64_parity(name):
    x, sc, h2, sp, a, _ = case(name)
    note(f"sparsify fp64 {name}")
    h = imported(name)
    sph = P.h2_sparsify(h, P.H2_FP64)
    _check_plan(sph, sp)
    amax = np.abs(a).max()
    for t, q in sp.q.items():
        got = P.h2_sparse_export_q(sph, t, q.shape[0])
        assert np.abs(got - q).max() <= 1e-12, f"Q of cluster {t}"
    worst = 0.0
    for (t, s), blk in sp.s_blocks.items():
        got = P.h2_sparse_export_block(sph, t, s, *blk.shape)
        worst = max(worst, np.abs(got - blk).max())
    assert worst <= 1e-12 * amax


@pytest.mark.parametrize("name", ["square1k", "cube1536", "cube2500r48"])
def test_sparsify_mixed_parity(name):
    x, sc, h2, sp, a, _ = case(name)
    note(f"sparsify mixed {name}")
    h = imported(name)
    sph = P.h2_sparsify(h, P.H2_MIXED)
    _check_plan(sph, sp)
    amax = np.abs(a).max()
    worst = 0.0
    for (t, s), blk in sp.s_blocks.items():
        got = P.h2_sparse_export_block(sph, t, s, *blk.shape)
        worst = max(worst, np.abs(got - blk).max())
    assert worst <= 5e-6 * amax


@pytest.mark.parametrize("name", list(CASES))
def test_preconditioner_matches_oracle_ilu0(name):
    x, sc, h2, sp, a, _ = case(name)
    note(f"apply inverse fp64 {name}")
    h = imported(name)
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_FP64))
    b = np.random.default_rng(3).standard_normal((x.shape[0], 2))
    out = dev(np.zeros_like(b))
    P.h2_apply_inverse(f, dev(b), out)
    ilu = oracle.BlockILU0(sp, oracle.elimination_order(sp))
    bt = to_tree(b, h2.tree.perm)
    want_t = oracle.apply_v(sp, ilu.solve(oracle.apply_ut(sp, bt)))
    want = from_tree(want_t, h2.tree.perm)
    assert np.abs(host(out) - want).max() <= 1e-10 * np.abs(want).max()


@pytest.mark.parametrize("name", ["cube2500r48", "sphere2k", "hodlr700"])
def test_split_schur_targets_match_oracle_ilu0(name, monkeypatch):
    """Long Schur sums cut into parts (forced with a tiny part size) still give
    the oracle's block ILU(0)."""
    x, sc, h2, sp, a, _ = case(name)
    note(f"apply inverse fp64 split-K {name}")
    monkeypatch.setenv("H2SP_SCHUR_SPLIT_K", "4")
    h = imported(name)
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_FP64))
    assert P.h2_last_work()[7] > 0
    b = np.random.default_rng(7).standard_normal((x.shape[0], 3))
    out = dev(np.zeros_like(b))
    P.h2_apply_inverse(f, dev(b), out)
    ilu = oracle.BlockILU0(sp, oracle.elimination_order(sp))
    bt = to_tree(b, h2.tree.perm)
    want = from_tree(oracle.apply_v(sp, ilu.solve(oracle.apply_ut(sp, bt))), h2.tree.perm)
    assert np.abs(host(out) - want).max() <= 1e-10 * np.abs(want).max()


def test_split_schur_targets_mixed_solve(monkeypatch):
    x, sc, h2, sp, a, (leaf, cheb, tol, cap, eta) = case("cube2500r48")
    note("solve mixed split-K cube2500r48")
    monkeypatch.setenv("H2SP_SCHUR_SPLIT_K", "4")
    h = P.h2_build(x, sc, 1.0, leaf, cheb, tol, cap, eta)
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_MIXED))
    assert P.h2_last_work()[7] > 0
    b = np.random.default_rng(8).standard_normal((x.shape[0], 4))
    xs = dev(np.zeros_like(b))
    info = P.h2_solve(f, dev(b), xs, tol=1e-10, max_iter=40)
    assert info["residual"] <= 1e-10
    ref = from_tree(np.linalg.solve(a, to_tree(b, h2.tree.perm)), h2.tree.perm)
    assert np.abs(host(xs) - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("split_k", [None, "4"], ids=["whole", "splitk"])
@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
def test_schur_tile_order_changes_no_bit(precision, split_k, monkeypatch):
    """Schur tiles ordered by Z position (forced on every level) give the same
    factor, bit for bit, as target order: each tile writes its own block."""
    x, sc, h2, sp, a, _ = case("cube2500r48")
    note(f"schur tile order precision={precision} split_k={split_k}")
    if split_k:
        monkeypatch.setenv("H2SP_SCHUR_SPLIT_K", split_k)
    h = imported("cube2500r48")
    b = np.random.default_rng(9).standard_normal((x.shape[0], 2))
    outs = []
    for order in ("0", "2"):
        monkeypatch.setenv("H2SP_SCHUR_ORDER", order)
        f = P.h2_factor_S(P.h2_sparsify(h, precision))
        if split_k:
            assert P.h2_last_work()[7] > 0
        out = dev(np.zeros_like(b))
        P.h2_apply_inverse(f, dev(b), out)
        outs.append(host(out))
    assert np.isfinite(outs[0]).all()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("name", list(CASES))
def test_exact_factor_fill_and_inverse(name):
    """Exact mode: the filled pattern matches the oracle's graph elimination
    bit for bit, and one application of V (L D L^T)^{-1} U^T is A_H2^{-1}."""
    x, sc, h2, sp, a, _ = case(name)
    note(f"exact factor fp64 {name}")
    h = imported(name)
    sph = P.h2_sparsify(h, P.H2_FP64)
    entries, flops = P.h2_factor_analyze(sph)
    f = P.h2_factor_S(sph, P.H2_FACTOR_EXACT)
    work = P.h2_last_work()
    assert work[9] == entries and abs(work[5] - flops) <= 1e-9 * max(flops, 1.0)
    plan = P.h2_sparse_export_plan(sph)
    order = oracle.elimination_order(sp)
    pos = {c: i for i, c in enumerate(order)}
    got = set()
    for i, t in enumerate(plan["elim"]):
        for b in range(plan["rowptr"][i], plan["rowptr"][i + 1]):
            got.add((int(t), int(plan["colidx"][b])))
    want = {(t, s) for (t, s) in oracle.block_fill(sp, order) if pos[t] <= pos[s]}
    assert got == want
    assert P.h2_last_work()[9] == sum(sp.nonbasis[t] * sp.nonbasis[s] for (t, s) in want)
    b = np.random.default_rng(10).standard_normal((x.shape[0], 3))
    out = dev(np.zeros_like(b))
    P.h2_apply_inverse(f, dev(b), out)
    ref = from_tree(np.linalg.solve(a, to_tree(b, h2.tree.perm)), h2.tree.perm)
    assert np.abs(host(out) - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["cube1536", "cube2500r48", "torus777"])
def test_exact_factor_mixed_solve(name):
    x, sc, h2, sp, a, (leaf, cheb, tol, cap, eta) = case(name)
    note(f"exact factor mixed {name}")
    h = P.h2_build(x, sc, 1.0, leaf, cheb, tol, cap, eta)
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_MIXED), P.H2_FACTOR_EXACT)
    b = np.random.default_rng(11).standard_normal((x.shape[0], 4))
    xs = dev(np.zeros_like(b))
    info = P.h2_solve(f, dev(b), xs, tol=1e-10, max_iter=10)
    assert info["residual"] <= 1e-10 and info["iters"] <= 3
    ref = from_tree(np.linalg.solve(a, to_tree(b, h2.tree.perm)), h2.tree.perm)
    assert np.abs(host(xs) - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("mode", ["exact", "ilu0"])
@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
def test_schur_merged_runs_match_per_pivot(precision, mode, monkeypatch):
    """Runs of pivots merged into one Schur segment (k-outer tiles, S copies in
    column order) and one segment per pivot give the same factor up to the
    grouping of the sums inside the MFMA steps, and the same Schur flops (the
    padding rows between merged pivots are not counted)."""
    name = "cube2500r48"
    x, sc, h2, sp, a, _ = case(name)
    note(f"schur merged runs {mode} precision={precision}")
    h = imported(name)
    fm = P.H2_FACTOR_EXACT if mode == "exact" else P.H2_FACTOR_ILU0
    b = np.random.default_rng(12).standard_normal((x.shape[0], 3))
    outs, flops = [], []
    for merge in ("0", "1"):
        monkeypatch.setenv("H2SP_SCHUR_MERGE", merge)
        f = P.h2_factor_S(P.h2_sparsify(h, precision), fm)
        flops.append(P.h2_last_work()[5])
        out = dev(np.zeros_like(b))
        P.h2_apply_inverse(f, dev(b), out)
        outs.append(host(out))
    assert np.isfinite(outs[0]).all() and np.isfinite(outs[1]).all()
    assert abs(flops[0] - flops[1]) <= 1e-12 * flops[0]
    bar = 1e-12 if precision == P.H2_FP64 else 1e-4
    assert np.abs(outs[0] - outs[1]).max() <= bar * np.abs(outs[0]).max()
    if mode == "exact" and precision == P.H2_FP64:
        ref = from_tree(np.linalg.solve(a, to_tree(b, h2.tree.perm)), h2.tree.perm)
        assert np.abs(outs[1] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_factor_twice_is_rejected():
    x, sc, h2, sp, a, _ = case("torus777")
    note("factor twice")
    sph = P.h2_sparsify(imported("torus777"), P.H2_FP64)
    P.h2_factor_S(sph)
    with pytest.raises(P.H2Error) as e:
        P.h2_factor_S(sph, P.H2_FACTOR_EXACT)
    assert e.value.code == P.H2_EINVAL


@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_solve_refined(name, precision):
    x, sc, h2, sp, a, (leaf, cheb, tol, cap, eta) = case(name)
    note(f"solve {name} precision={precision}")
    h = P.h2_build(x, sc, 1.0, leaf, cheb, tol, cap, eta)
    f = P.h2_factor_S(P.h2_sparsify(h, precision))
    b = np.random.default_rng(4).standard_normal((x.shape[0], 5))
    xs = dev(np.zeros_like(b))
    info = P.h2_solve(f, dev(b), xs, tol=1e-10, max_iter=40)
    assert info["residual"] <= 1e-10
    ref = from_tree(np.linalg.solve(a, to_tree(b, h2.tree.perm)), h2.tree.perm)
    assert np.abs(host(xs) - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("n", [1, 2, 30, 65])
def test_tiny_and_single_leaf(n):
    note(f"tiny n={n}")
    x, sc, h2 = make_case("cube", n, 21, 32, 3)
    h = P.h2_build(x, sc, 1.0, 32, 3)
    sph = P.h2_sparsify(h, P.H2_FP64)
    f = P.h2_factor_S(sph)
    b = np.random.default_rng(5).standard_normal((n, 1))
    xs = dev(np.zeros_like(b))
    P.h2_solve(f, dev(b), xs, tol=1e-12)
    a = h2.dense()
    ref = from_tree(np.linalg.solve(a, to_tree(b, h2.tree.perm)), h2.tree.perm)
    assert np.abs(host(xs) - ref).max() <= 1e-10 * np.abs(ref).max()


def test_many_rhs_cross_tiles():
    x, sc, h2, sp, a, (leaf, cheb, tol, cap, eta) = case("cube1536")
    note("solve nrhs=33")
    h = P.h2_build(x, sc, 1.0, leaf, cheb, tol, cap, eta)
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_MIXED))
    b = np.random.default_rng(6).standard_normal((x.shape[0], 33))
    xs = dev(np.zeros_like(b))
    P.h2_solve(f, dev(b), xs, tol=1e-10)
    ref = from_tree(np.linalg.solve(a, to_tree(b, h2.tree.perm)), h2.tree.perm)
    assert np.abs(host(xs) - ref).max() <= 1e-8 * np.abs(ref).max()


def test_fp64_sparsify_is_deterministic():
    x, sc, h2, sp, a, _ = case("cube2500r48")
    note("determinism")
    h = imported("cube2500r48")
    s1 = P.h2_sparsify(h, P.H2_FP64)
    s2 = P.h2_sparsify(h, P.H2_FP64)
    plan = P.h2_sparse_export_plan(s1)
    for i, t in enumerate(plan["elim"][:200]):
        for b in range(plan["rowptr"][i], plan["rowptr"][i + 1]):
            s = int(plan["colidx"][b])
            m1, m2 = sp.nonbasis[t], sp.nonbasis[s]
            assert np.array_equal(P.h2_sparse_export_block(s1, t, s, m1, m2),
                                  P.h2_sparse_export_block(s2, t, s, m1, m2))


BATCH = ["cube1536", "sphere2k", "torus777", "cube2500r48", "hodlr700", "square1k"]


@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
def test_sparsify_batch_matches_single(precision):
    """One merged level sweep over instances of different size, depth, rank,
    admissibility and dimension gives every instance exactly its own result."""
    note(f"sparsify batch precision={precision}")
    hs = [imported(n) for n in BATCH]
    batch = P.h2_sparsify_batch(hs, precision)
    for name, h, spb in zip(BATCH, hs, batch):
        sp = case(name)[3]
        single = P.h2_sparsify(imported(name), precision)
        _check_plan(spb, sp)
        for t, q in sp.q.items():
            assert np.array_equal(P.h2_sparse_export_q(spb, t, q.shape[0]),
                                  P.h2_sparse_export_q(single, t, q.shape[0])), f"{name}: Q of {t}"
        for (t, s), blk in sp.s_blocks.items():
            got = P.h2_sparse_export_block(spb, t, s, *blk.shape)
            assert np.array_equal(got, P.h2_sparse_export_block(single, t, s, *blk.shape)), f"{name}: S {t},{s}"


def test_factor_solve_batch():
    note("factor + solve batch mixed")
    hs = [P.h2_build(case(n)[0], case(n)[1], 1.0, *case(n)[5]) for n in BATCH]
    sps = P.h2_sparsify_batch(hs, P.H2_MIXED)
    fs = P.h2_factor_S_batch(sps)
    rng = np.random.default_rng(12)
    bs, xs, refs = [], [], []
    for i, name in enumerate(BATCH):
        x, sc, h2, sp, a, _ = case(name)
        b = rng.standard_normal((x.shape[0], 1 + i))
        bs.append(dev(b))
        xs.append(dev(np.zeros_like(b)))
        refs.append(from_tree(np.linalg.solve(a, to_tree(b, h2.tree.perm)), h2.tree.perm))
    infos = P.h2_solve_batch(fs, bs, xs, tol=1e-10, max_iter=40)
    for name, info, xv, ref, b in zip(BATCH, infos, xs, refs, bs):
        assert info["residual"] <= 1e-10, name
        assert np.abs(host(xv) - ref).max() <= 1e-8 * np.abs(ref).max(), name
    # the same instance alone gives the same bits
    h0 = P.h2_build(case(BATCH[1])[0], case(BATCH[1])[1], 1.0, *case(BATCH[1])[5])
    f0 = P.h2_factor_S(P.h2_sparsify(h0, P.H2_MIXED))
    x0 = dev(np.zeros((case(BATCH[1])[0].shape[0], 2)))
    P.h2_solve(f0, bs[1], x0, tol=1e-10, max_iter=40)
    assert np.array_equal(host(x0), host(xs[1]))


def test_batch_rejects_repeated_handles():
    note("batch argument errors")
    sp = P.h2_sparsify(imported("torus777"), P.H2_FP64)
    with pytest.raises(P.H2Error) as e:
        P.h2_factor_S_batch([sp, sp])
    assert e.value.code == P.H2_EINVAL
    # one matrix twice: its device copy and its matvec plan are per matrix
    h = imported("torus777")
    with pytest.raises(P.H2Error) as e:
        P.h2_sparsify_batch([h, h], P.H2_FP64)
    assert e.value.code == P.H2_EINVAL
    f1 = P.h2_factor_S(P.h2_sparsify(h, P.H2_FP64))
    f2 = P.h2_factor_S(P.h2_sparsify(h, P.H2_MIXED))
    b = dev(np.ones((777, 1)))
    xs = [dev(np.zeros((777, 1))), dev(np.zeros((777, 1)))]
    with pytest.raises(P.H2Error) as e:
        P.h2_solve_batch([f1, f2], [b, b], xs, tol=1e-10)
    assert e.value.code == P.H2_EINVAL


def test_graph_replays_match_eager(tmp_path):
    """The captured preconditioner and matvec, replayed three times with other
    work in between, give exactly what the eager launches give (a child
    process with graphs off) and the oracle's results."""
    import os
    import subprocess
    from graph_cases import run_sequence
    note("graph replays vs eager")
    got = run_sequence(P)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = tmp_path / "eager.npy"
    env = dict(os.environ, H2SP_GRAPHS="0")
    subprocess.run([sys.executable, os.path.join(root, "tests", "graph_child.py"), root, str(out)],
                   env=env, check=True, timeout=300)
    eager = np.load(out)
    assert np.array_equal(got, eager)
    # and against the oracle: the matvec replays are A_H2 b
    x, sc, h2, sp, a, _ = case("cube1536")
    rng = np.random.default_rng(21)
    for rep in range(3):
        b = rng.standard_normal((1536, 3))
        want = from_tree(a @ to_tree(b, h2.tree.perm), h2.tree.perm)
        assert np.abs(got[2 * rep + 1] - want).max() <= 1e-10 * np.abs(want).max()
