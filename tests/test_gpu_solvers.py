"""GPU tests of the solve methods and of the error paths (through the C ABI).

* flexible GMRES (H2_SOLVE_GMRES) against the dense solve of A_H2;
* the automatic fallback: on an indefinite exp-core matrix (diagonal value
  1.02, so 0.02 I plus a Gaussian Gram matrix, made slightly indefinite by the
  far-field approximation: its smallest eigenvalue is about -0.03) the block
  ILU(0) refinement diverges (residual 0.85, then 12, ...: the oracle's
  refinement shows it), the solver goes back to the best x and GMRES reaches
  the tolerance (the oracle's GMRES needs about 26 steps);
* h2_solve_with: an accurate H^2 matrix solved with the factor of a coarser
  one of the same points as preconditioner;
* H2_ENOCONV: x is still written and the info filled;
* H2_ESINGULAR: an exactly singular pivot block (two points at distance 1,
  kernel 1/r, diagonal 1: the block [[1, 1], [1, 1]]) is reported by the
  host, with no device fault.
Bars: the true relative residual ||b - A x|| / ||b|| from the dense matrix,
and x within 1e-8 of the dense solve where A is well conditioned.
"""

import sys

import numpy as np
import pytest

import h2inputs
import oracle
import paper_1705_04601_amd as P
from h2test_util import import_arrays, make_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def note(msg):
    sys.stderr.write(f"[gpu-case] {msg}\n")
    sys.stderr.flush()


def dev(arr):
    arr = np.asarray(arr, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(arr.T)).cuda().T


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def from_tree(v_tree, perm):
    out = np.empty_like(v_tree)
    out[perm] = v_tree
    return out


_cache = {}


def invdist_case():
    if "inv" not in _cache:
        x, sc, h2 = make_case("cube", 1536, 11, 32, 3, 1e-8, 27)
        h = P.h2_import(x, sc, 1.0, 32, 3, 1.0, *import_arrays(h2))
        _cache["inv"] = (x, sc, h2, h2.dense(), h)
    return _cache["inv"]


def exp_indefinite_case():
    if "exp" not in _cache:
        x = h2inputs.points("cube", 1536, 11)
        h2 = oracle.build_h2(x, 32, 3, 1.0, 1.02, 1e-8, 27, 1.0, oracle.EXP)
        h = P.h2_import(x, 1.0, 1.02, 32, 3, 1.0, *import_arrays(h2), kernel=P.H2_KERNEL_EXP)
        _cache["exp"] = (x, h2, h2.dense(), h)
    return _cache["exp"]


@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
def test_gmres_matches_dense_solve(precision):
    note(f"gmres invdist precision={precision}")
    x, sc, h2, a, h = invdist_case()
    f = P.h2_factor_S(P.h2_sparsify(h, precision))
    b = np.random.default_rng(41).standard_normal((1536, 3))
    xs = dev(np.zeros_like(b))
    info = P.h2_solve(f, dev(b), xs, tol=1e-10, max_iter=40, method=P.H2_SOLVE_GMRES, restart=8)
    assert info["gmres_steps"] == info["iters"] and info["refine_steps"] == 0
    assert info["residual"] <= 1e-10
    perm = h2.tree.perm
    got = host(xs)
    true_res = np.linalg.norm(b[perm] - a @ got[perm], axis=0) / np.linalg.norm(b, axis=0)
    assert true_res.max() <= 2e-10
    ref = from_tree(np.linalg.solve(a, b[perm]), perm)
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
def test_refinement_falls_back_to_gmres(precision):
    note(f"auto solve, diverging refinement precision={precision}")
    x, h2, a, h = exp_indefinite_case()
    f = P.h2_factor_S(P.h2_sparsify(h, precision))
    b = np.random.default_rng(42).standard_normal((1536, 2))
    xs = dev(np.zeros_like(b))
    info = P.h2_solve(f, dev(b), xs, tol=1e-10, max_iter=80)
    note(f"  refine {info['refine_steps']} gmres {info['gmres_steps']} residual {info['residual']:.2e}")
    assert info["refine_steps"] >= 2 and info["gmres_steps"] > 0
    assert info["residual"] <= 1e-10
    perm = h2.tree.perm
    got = host(xs)
    true_res = np.linalg.norm(b[perm] - a @ got[perm], axis=0) / np.linalg.norm(b, axis=0)
    assert true_res.max() <= 2e-10
    # refinement alone diverges on this matrix
    xr = dev(np.zeros_like(b))
    info_r = P.h2_solve(f, dev(b), xr, tol=1e-10, max_iter=6, method=P.H2_SOLVE_REFINE, check=False)
    assert info_r["code"] == P.H2_ENOCONV and info_r["gmres_steps"] == 0
    assert not (info_r["residual"] <= 1.0)


def test_solve_with_a_coarser_preconditioner():
    """A accurate (Chebyshev 4, 1e-10); the preconditioner is the factor of a
    Chebyshev 2 H^2 matrix of the same points (Section 5.5's setup)."""
    note("solve_with fine operator, coarse factor")
    x = h2inputs.points("cube", 1536, 11)
    sc = 1.0 / (4 * np.pi * 1536)
    fine = oracle.build_h2(x, 32, 4, sc, 1.0, 1e-10, 64, 1.0)
    coarse = oracle.build_h2(x, 32, 2, sc, 1.0, 0.0, 0, 1.0)
    hf = P.h2_import(x, sc, 1.0, 32, 4, 1.0, *import_arrays(fine))
    hc = P.h2_import(x, sc, 1.0, 32, 2, 1.0, *import_arrays(coarse))
    f = P.h2_factor_S(P.h2_sparsify(hc, P.H2_MIXED))
    b = np.random.default_rng(43).standard_normal((1536, 2))
    xs = dev(np.zeros_like(b))
    info = P.h2_solve_with(hf, f, dev(b), xs, tol=1e-10, max_iter=60)
    assert info["residual"] <= 1e-10 and info["gmres_steps"] > 0
    a = fine.dense()
    perm = fine.tree.perm
    ref = from_tree(np.linalg.solve(a, b[perm]), perm)
    assert np.abs(host(xs) - ref).max() <= 1e-8 * np.abs(ref).max()
    # different points: refused
    other = P.h2_build(h2inputs.points("cube", 1536, 12), sc, 1.0, 32, 2)
    with pytest.raises(P.H2Error) as e:
        P.h2_solve_with(other, f, dev(b), xs, tol=1e-10)
    assert e.value.code == P.H2_EINVAL


def test_enoconv_writes_x_and_info():
    note("ENOCONV")
    x, sc, h2, a, h = invdist_case()
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_MIXED))
    b = np.random.default_rng(44).standard_normal((1536, 2))
    xs = dev(np.zeros_like(b))
    with pytest.raises(P.H2Error) as e:
        P.h2_solve(f, dev(b), xs, tol=1e-30, max_iter=2)
    assert e.value.code == P.H2_ENOCONV
    info = P.h2_solve(f, dev(b), xs, tol=1e-30, max_iter=2, check=False)
    assert info["code"] == P.H2_ENOCONV and info["iters"] == 2
    assert 0 < info["residual"] <= 1e-6
    perm = h2.tree.perm
    ref = from_tree(np.linalg.solve(a, b[perm]), perm)
    assert np.abs(host(xs) - ref).max() <= 1e-6 * np.abs(ref).max()


@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
def test_esingular_pivot_block(precision):
    note(f"ESINGULAR precision={precision}")
    pts = np.array([[0.0, 0.0], [1.0, 0.0]])
    h = P.h2_build(pts, 1.0, 1.0, 32, 2)
    sp = P.h2_sparsify(h, precision)
    with pytest.raises(P.H2Error) as e:
        P.h2_factor_S(sp)
    assert e.value.code == P.H2_ESINGULAR
    assert "singular" in str(e.value)
    # the device is still usable afterwards
    x, sc, h2, a, hh = invdist_case()
    v = np.ones((1536, 1))
    y = dev(np.zeros_like(v))
    P.h2_matvec(hh, dev(v), y)
    assert np.isfinite(host(y)).all()


def test_solve_option_errors():
    note("solve option errors")
    x, sc, h2, a, h = invdist_case()
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_FP64))
    b = dev(np.ones((1536, 1)))
    xs = dev(np.zeros((1536, 1)))
    for kw in (dict(method=7), dict(restart=65)):
        with pytest.raises(P.H2Error) as e:
            P.h2_solve(f, b, xs, **kw)
        assert e.value.code == P.H2_EINVAL
