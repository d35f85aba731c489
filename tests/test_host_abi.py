"""CPU tests of the library boundary: symbols, argument checks, host planning.

The tree, the block tree and the rank decisions of the library's host code
are compared bit for bit with the oracle (independent implementations).
No device work is started here.
"""

import ctypes

import numpy as np
import pytest

import paper_1705_04601_amd as P
from h2test_util import make_case


def test_library_exports_every_header_symbol():
    lib = P.lib()
    names = P.header_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("kind,n,seed,leaf,cheb,tol,cap,eta", [
    ("square", 1024, 1, 32, 4, 0.0, 16, 1.0),
    ("sphere", 4096, 2, 64, 3, 1e-8, 27, 1.0),
    ("cube", 3000, 3, 32, 3, 1e-8, 27, 1.0),
    ("torus", 777, 13, 24, 3, 1e-8, 20, 1.0),
    ("cube", 2500, 8, 40, 4, 1e-8, 48, 1.0),
    ("square", 700, 9, 16, 4, 0.0, 16, 0.0),
    ("cube", 5, 9, 32, 3, 0.0, 0, 1.0),
])
def test_tree_and_ranks_match_oracle(kind, n, seed, leaf, cheb, tol, cap, eta):
    x, sc, h2 = make_case(kind, n, seed, leaf, cheb, tol, cap, eta)
    h = P.h2_build(x, sc, 1.0, leaf, cheb, tol, cap, eta)
    depth, ncl, npts = P.h2_matrix_info(h)
    assert depth == h2.tree.depth and ncl == h2.tree.ncl and npts == cheb ** x.shape[1]
    perm, rank = P.h2_matrix_export_tree(h, n)
    assert np.array_equal(perm, h2.tree.perm)
    assert np.array_equal(rank, h2.rank)


@pytest.mark.parametrize("kind,n,seed,leaf,cheb,tol,cap", [
    ("cube", 2000, 21, 32, 4, 1e-8, 48),
    ("square", 1500, 22, 32, 4, 1e-8, 16),
    ("sphere", 2048, 12, 64, 3, 1e-6, 27),
])
def test_exp_kernel_tree_and_ranks_match_oracle(kind, n, seed, leaf, cheb, tol, cap):
    """The exp core of Example 5.2 through the library's host construction:
    permutation and recompressed ranks equal the oracle's."""
    import h2inputs
    import oracle
    x = h2inputs.points(kind, n, seed)
    h2 = oracle.build_h2(x, leaf, cheb, 1.0, 3.0, tol, cap, 1.0, oracle.EXP)
    h = P.h2_build(x, 1.0, 3.0, leaf, cheb, tol, cap, 1.0, kernel=P.H2_KERNEL_EXP)
    perm, rank = P.h2_matrix_export_tree(h, n)
    assert np.array_equal(perm, h2.tree.perm)
    assert np.array_equal(rank, h2.rank)


def _build_code(x, msgs=None, **kw):
    """Status of h2_build; the message of a failure goes to `msgs`, read
    right after the failing call (it is per thread and per call)."""
    args = dict(scale=1.0, diag=1.0, leaf=16, cheb=3, tol=0.0, rank_cap=0, eta=1.0)
    args.update(kw)
    try:
        P.h2_build(x, **args)
    except P.H2Error as e:
        if msgs is not None:
            msgs.append(P.lib().h2_last_error().decode())
        return e.code
    return P.H2_OK


def test_argument_errors():
    x = np.random.default_rng(0).random((100, 3))
    assert _build_code(x) == P.H2_OK
    bad = x.copy()
    bad[7, 1] = np.nan
    assert _build_code(bad) == P.H2_EINVAL
    dup = x.copy()
    dup[5] = dup[9]
    msgs = []
    assert _build_code(dup, msgs) == P.H2_EINVAL
    assert "duplicate" in msgs[0]
    assert _build_code(np.random.default_rng(0).random((10, 4))) == P.H2_EINVAL
    assert _build_code(x, leaf=1) == P.H2_EINVAL
    assert _build_code(x, leaf=129) == P.H2_EINVAL
    assert _build_code(x, cheb=5) == P.H2_EUNSUPPORTED
    assert _build_code(x, eta=-1.0) == P.H2_EINVAL
    assert _build_code(x, kernel=7) == P.H2_EUNSUPPORTED
    assert _build_code(x, kernel=P.H2_KERNEL_EXP, diag=3.0) == P.H2_OK


def test_null_handles_are_rejected():
    lib = P.lib()
    out = ctypes.c_void_p()
    assert lib.h2_sparsify(None, None, ctypes.byref(out)) == P.H2_EINVAL
    assert lib.h2_factor_S(None, None, ctypes.byref(out)) == P.H2_EINVAL
    assert lib.h2_matvec(None, None, None, 1, 1) == P.H2_EINVAL
    lib.h2_matrix_destroy(None)
    lib.h2_sparse_destroy(None)
    lib.h2_factor_destroy(None)


@pytest.mark.parametrize("d", [1e-3, 1e-2])
def test_ifmm_kernel_tree_and_ranks_match_oracle(d):
    """The Example 5.4 kernel of Section 5.5 through the library's host
    construction: permutation and recompressed ranks equal the oracle's."""
    import h2inputs
    import oracle
    x = h2inputs.points("cube", 1500, 41)
    h2 = oracle.build_h2(x, 32, 4, 1.0, 1.0, 1e-3, 64, 1.0, (oracle.IFMM, d))
    h = P.h2_build(x, 1.0, 1.0, 32, 4, 1e-3, 64, 1.0, kernel=P.H2_KERNEL_IFMM, param=d)
    perm, rank = P.h2_matrix_export_tree(h, 1500)
    assert np.array_equal(perm, h2.tree.perm)
    assert np.array_equal(rank, h2.rank)


def test_ifmm_kernel_needs_a_positive_d():
    x = np.random.default_rng(0).random((100, 3))
    with pytest.raises(P.H2Error) as e:
        P.h2_build(x, 1.0, 1.0, 32, 3, kernel=P.H2_KERNEL_IFMM, param=0.0)
    assert e.value.code == P.H2_EINVAL
