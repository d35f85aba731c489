"""GPU parity at the block shapes of the N = 1,048,576 workload (through the C ABI).

The largest workload (unit cube, leaf 128, Chebyshev 4^3 recompressed, ranks
<= 64, c = 1/(4 pi N)) runs clusters of 128 points, leaf bases of up to 64
columns, father bases of 128 x 64 and pivot blocks of 128 x 128.  The two
cases here reproduce those shapes at N = 8192 (64 leaves of 128 points), where
the oracle still finishes in seconds:

  * cube8k_c5: the same recipe (tolerance 1e-8, cap 64); ranks up to 53;
  * cube8k_r64: tolerance 1e-12 so that the cap binds: 48 clusters of rank 64,
    so leaves keep k_t = 64 of their 128 rows, the Householder QR runs at
    n = 128, r = 64 (four 32-column chunks of Q) and the top clusters have
    m = 128 rows.

Bars (each written in its test):
  * sizes, S offsets, elimination order, S block pattern: bit-exact;
  * FP64: Q_t within 1e-12, S blocks within 1e-12 max|A|, matvec within 1e-13,
    one application of V (L D L^T)^{-1} U^T within 1e-10 of the oracle's
    block ILU(0);
  * mixed: S blocks within 5e-6 max|A| and the preconditioner application
    within the FP32 bar derived in test_preconditioner_mixed;
  * refined solves: relative residual <= 1e-10, x within 1e-8 of the dense
    solve of A_H2.
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
    "cube8k_c5": ("cube", 8192, 5, 128, 4, 1e-8, 64, 1.0),
    "cube8k_r64": ("cube", 8192, 5, 128, 4, 1e-12, 64, 1.0),
}
_cache = {}


def note(msg):
    sys.stderr.write(f"[gpu-case] {msg}\n")
    sys.stderr.flush()


def case(name):
    if name not in _cache:
        kind, n, seed, leaf, cheb, tol, cap, eta = CASES[name]
        x, sc, h2 = make_case(kind, n, seed, leaf, cheb, tol, cap, eta)
        sp = oracle.sparsify(h2)
        _cache[name] = {"x": x, "sc": sc, "h2": h2, "sp": sp, "opts": (leaf, cheb, tol, cap, eta)}
    return _cache[name]


def dense(name):
    c = case(name)
    if "a" not in c:
        c["a"] = c["h2"].dense()
    return c["a"]


def ilu(name):
    c = case(name)
    if "ilu" not in c:
        sp = c["sp"]
        c["ilu"] = oracle.BlockILU0(sp, oracle.elimination_order(sp))
    return c["ilu"]


def dev(arr):
    arr = np.asarray(arr, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(arr.T)).cuda().T


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def imported(name):
    c = case(name)
    leaf, cheb, tol, cap, eta = c["opts"]
    return P.h2_import(c["x"], c["sc"], 1.0, leaf, cheb, eta, *import_arrays(c["h2"]))


def from_tree(v_tree, perm):
    out = np.empty_like(v_tree)
    out[perm] = v_tree
    return out


def oracle_preconditioner(name, b):
    c = case(name)
    sp, perm = c["sp"], c["h2"].tree.perm
    return from_tree(oracle.apply_v(sp, ilu(name).solve(oracle.apply_ut(sp, b[perm]))), perm)


@pytest.mark.parametrize("name", list(CASES))
def test_shapes_reach_the_large_workload(name):
    """The cases do reach the shapes they stand for (a host-side check of the
    oracle's plan, so that a change of inputs cannot silently shrink them)."""
    c = case(name)
    sp, h2 = c["sp"], c["h2"]
    assert sp.n_act.max() == 128 and sp.nonbasis.max() == 128
    assert (h2.tree.size[h2.tree.ncl // 2:] == 128).all()
    if name == "cube8k_r64":
        assert (sp.kept == 64).sum() >= 32
        assert any(q.shape[0] == 128 and sp.kept[t] == 64 for t, q in sp.q.items())


def _check_plan(sph, sp):
    plan = P.h2_sparse_export_plan(sph)
    for key in ("n_act", "kept", "nonbasis", "soff"):
        assert np.array_equal(plan[key], getattr(sp, key)), key
    elim = [int(c) for c in plan["elim"] if sp.nonbasis[c] > 0]
    assert elim == oracle.elimination_order(sp)
    pos = {int(c): i for i, c in enumerate(plan["elim"])}
    got = set()
    for i, t in enumerate(plan["elim"]):
        for b in range(plan["rowptr"][i], plan["rowptr"][i + 1]):
            got.add((int(t), int(plan["colidx"][b])))
    assert got == {(t, s) for (t, s) in sp.s_blocks if pos[t] <= pos[s]}


@pytest.mark.parametrize("name", list(CASES))
def test_matvec(name):
    note(f"c5-shape matvec {name}")
    c = case(name)
    a, perm = dense(name), c["h2"].tree.perm
    v = np.random.default_rng(31).standard_normal((8192, 3))
    y = dev(np.zeros_like(v))
    P.h2_matvec(imported(name), dev(v), y)
    want = from_tree(a @ v[perm], perm)
    assert np.abs(host(y) - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("name", list(CASES))
def test_sparsify_fp64(name):
    note(f"c5-shape sparsify fp64 {name}")
    c = case(name)
    sp = c["sp"]
    sph = P.h2_sparsify(imported(name), P.H2_FP64)
    _check_plan(sph, sp)
    for t, q in sp.q.items():
        got = P.h2_sparse_export_q(sph, t, q.shape[0])
        assert np.abs(got - q).max() <= 1e-12, f"Q of cluster {t} ({q.shape[0]} x {q.shape[0]})"
    amax = np.abs(dense(name)).max()
    worst = max(np.abs(P.h2_sparse_export_block(sph, t, s, *blk.shape) - blk).max()
                for (t, s), blk in sp.s_blocks.items())
    assert worst <= 1e-12 * amax


@pytest.mark.parametrize("name", list(CASES))
def test_sparsify_mixed(name):
    note(f"c5-shape sparsify mixed {name}")
    c = case(name)
    sp = c["sp"]
    sph = P.h2_sparsify(imported(name), P.H2_MIXED)
    _check_plan(sph, sp)
    amax = np.abs(dense(name)).max()
    worst = max(np.abs(P.h2_sparse_export_block(sph, t, s, *blk.shape) - blk).max()
                for (t, s), blk in sp.s_blocks.items())
    assert worst <= 5e-6 * amax


@pytest.mark.parametrize("name", list(CASES))
def test_preconditioner_fp64(name):
    note(f"c5-shape apply inverse fp64 {name}")
    f = P.h2_factor_S(P.h2_sparsify(imported(name), P.H2_FP64))
    b = np.random.default_rng(32).standard_normal((8192, 3))
    out = dev(np.zeros_like(b))
    P.h2_apply_inverse(f, dev(b), out)
    want = oracle_preconditioner(name, b)
    assert np.abs(host(out) - want).max() <= 1e-10 * np.abs(want).max()


@pytest.mark.parametrize("name", list(CASES))
def test_preconditioner_mixed(name):
    """FP32 sparsification, factorisation and triangular solves against the
    oracle's FP64 block ILU(0).  Bar: each FP32 dot product of the transforms
    (two products over at most 2 x 128 terms per level) errs by at most about
    2 (2 n_max) u32 relative to the block, u32 = 2^-24, n_max = 128, i.e.
    3.1e-5; the factor and the solves add products of the same length and
    the preconditioned operator's condition number (about 1.2 for this
    kernel) multiplies it: 4 x 3.1e-5 = 1.2e-4 relative to max |x|."""
    note(f"c5-shape apply inverse mixed {name}")
    f = P.h2_factor_S(P.h2_sparsify(imported(name), P.H2_MIXED))
    b = np.random.default_rng(33).standard_normal((8192, 2))
    out = dev(np.zeros_like(b))
    P.h2_apply_inverse(f, dev(b), out)
    want = oracle_preconditioner(name, b)
    u32 = 2.0 ** -24
    bar = 4 * 2 * (2 * 128) * u32
    err = np.abs(host(out) - want).max() / np.abs(want).max()
    note(f"  mixed preconditioner error {err:.3e} (bar {bar:.2e})")
    assert err <= bar


@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_solve_refined(name, precision):
    note(f"c5-shape solve {name} precision={precision}")
    c = case(name)
    f = P.h2_factor_S(P.h2_sparsify(imported(name), precision))
    b = np.random.default_rng(34).standard_normal((8192, 4))
    xs = dev(np.zeros_like(b))
    info = P.h2_solve(f, dev(b), xs, tol=1e-10, max_iter=20)
    assert info["residual"] <= 1e-10
    perm = c["h2"].tree.perm
    ref = from_tree(np.linalg.solve(dense(name), b[perm]), perm)
    assert np.abs(host(xs) - ref).max() <= 1e-8 * np.abs(ref).max()
