"""GPU tests of the preconditioner variant of Section 5.5 (through the C ABI):
the Example 5.4 kernel (H2_KERNEL_IFMM), the block threshold ILU of S
(H2_FACTOR_ILUT) and GMRES on an accurate H^2 matrix preconditioned by the
factor of a coarse one.

Setup of Section 5.5 at N = 1500 (random points in the unit cube, d = 1e-3
and 1e-2): the accurate H^2 matrix recompressed to 1e-9, the coarse one to
1e-3, both built by the oracle and imported, so that both sides work on the
same matrices.  Bars:
  * the S block pattern bit-exact and S within 1e-12 of the oracle (FP64);
  * one application of V (ILUt)^{-1} U^T within 1e-10 of the oracle's
    symmetric block ILUt (oracle.SymBlockILUT), and the numbers of fill
    blocks dropped and kept equal to the oracle's, at tau = inf (block
    ILU(0): also equal to H2_FACTOR_ILU0 within 1e-12), at a tau that keeps
    part of the fill, and at tau = 0 (the exact factor: within 1e-10 of the
    dense solve of S);
  * GMRES (FP64 and mixed factor) to a relative residual of 1e-10 of the
    accurate matrix, x within 1e-7 of its dense solve (cond up to about 4e3
    at d = 1e-2), in at most 20 steps.
"""

import sys

import numpy as np
import pytest

import h2inputs
import oracle
import paper_1705_04601_amd as P
from h2test_util import import_arrays
from test_gpu_parity import _check_plan

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 1500
D = (1e-3, 1e-2)
_cache = {}


def note(msg):
    sys.stderr.write(f"[gpu-case] {msg}\n")
    sys.stderr.flush()


def dev(arr):
    arr = np.asarray(arr, dtype=np.float64)
    return torch.from_numpy(np.ascontiguousarray(arr.T)).cuda().T


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def to_tree(v, perm):
    return v[perm]


def from_tree(v_tree, perm):
    out = np.empty_like(v_tree)
    out[perm] = v_tree
    return out


def case(d):
    if d not in _cache:
        x = h2inputs.points("cube", N, 41)
        kern = (oracle.IFMM, d)
        fine = oracle.build_h2(x, 32, 4, 1.0, 1.0, 1e-9, 64, 1.0, kern)
        coarse = oracle.build_h2(x, 32, 4, 1.0, 1.0, 1e-3, 64, 1.0, kern)
        sp = oracle.sparsify(coarse)
        order = oracle.elimination_order(sp)
        imp = lambda h2: P.h2_import(x, 1.0, 1.0, 32, 4, 1.0, *import_arrays(h2),
                                     kernel=P.H2_KERNEL_IFMM, param=d)
        _cache[d] = dict(x=x, fine=fine, coarse=coarse, sp=sp, order=order, hf=imp(fine), hc=imp(coarse))
    return _cache[d]


@pytest.mark.parametrize("d", D)
def test_ifmm_matvec_matches_oracle(d):
    note(f"ifmm matvec d={d}")
    c = case(d)
    v = np.random.default_rng(1).standard_normal((N, 2))
    y = dev(np.zeros_like(v))
    P.h2_matvec(c["hf"], dev(v), y)
    perm = c["fine"].tree.perm
    want = from_tree(c["fine"].matvec(to_tree(v, perm)), perm)
    assert np.abs(host(y) - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("d", D)
def test_ifmm_sparsified_s_matches_oracle(d):
    note(f"ifmm sparsify d={d}")
    c = case(d)
    sp = c["sp"]
    s = P.h2_sparsify(c["hc"], P.H2_FP64)
    _check_plan(s, sp)
    amax = max(np.abs(b).max() for b in sp.s_blocks.values())
    for (t, u), blk in sp.s_blocks.items():
        got = P.h2_sparse_export_block(s, t, u, sp.nonbasis[t], sp.nonbasis[u])
        assert np.abs(got - blk).max() <= 1e-12 * amax, (t, u)


@pytest.mark.parametrize("d,tau", [(1e-2, np.inf), (1e-2, 3e-5), (1e-2, 0.0), (1e-3, 1e-5)])
def test_ilut_application_matches_oracle(d, tau):
    note(f"ilut fp64 d={d} tau={tau}")
    c = case(d)
    sp, order = c["sp"], c["order"]
    f = P.h2_factor_S(P.h2_sparsify(c["hc"], P.H2_FP64), P.H2_FACTOR_ILUT, tau)
    work = P.h2_last_work()
    il = oracle.SymBlockILUT(sp, tau, order)
    assert (int(work[16]), int(work[17])) == (il.dropped, il.kept_fill)
    b = np.random.default_rng(5).standard_normal((N, 2))
    out = dev(np.zeros_like(b))
    P.h2_apply_inverse(f, dev(b), out)
    perm = c["coarse"].tree.perm
    bt = to_tree(b, perm)
    want = from_tree(oracle.apply_v(sp, il.solve(oracle.apply_ut(sp, bt))), perm)
    got = host(out)
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()
    if tau == np.inf:
        g0 = P.h2_factor_S(P.h2_sparsify(c["hc"], P.H2_FP64), P.H2_FACTOR_ILU0)
        out0 = dev(np.zeros_like(b))
        P.h2_apply_inverse(g0, dev(b), out0)
        assert np.abs(got - host(out0)).max() <= 1e-12 * np.abs(want).max()
    if tau == 0.0:
        assert il.dropped == 0
        ex = from_tree(oracle.apply_v(sp, np.linalg.solve(oracle.dense_s(sp), oracle.apply_ut(sp, bt))), perm)
        assert np.abs(got - ex).max() <= 1e-10 * np.abs(ex).max()


@pytest.mark.parametrize("tau", [3e-5, 1e-3, np.inf])
@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
def test_ilut_pruned_plans_match_full_fill(precision, tau, monkeypatch):
    """Planning each level without the blocks dropped so far (they hold zeros)
    gives the same drop decisions and the same factor, up to the grouping of
    the sums, as planning on the full structural fill, and less Schur work."""
    note(f"ilut pruned plans precision={precision} tau={tau}")
    c = case(1e-2)
    b = np.random.default_rng(6).standard_normal((N, 2))
    outs, counts, flops = [], [], []
    for prune in ("0", "1"):
        monkeypatch.setenv("H2SP_ILUT_PRUNE", prune)
        f = P.h2_factor_S(P.h2_sparsify(c["hc"], precision), P.H2_FACTOR_ILUT, tau)
        work = P.h2_last_work()
        counts.append((int(work[16]), int(work[17])))
        flops.append(work[5])
        out = dev(np.zeros_like(b))
        P.h2_apply_inverse(f, dev(b), out)
        outs.append(host(out))
    assert counts[0] == counts[1]
    if counts[0][0] > 0:
        assert flops[1] < flops[0]
    else:
        assert flops[1] == flops[0]
    bar = 1e-12 if precision == P.H2_FP64 else 1e-4
    assert np.isfinite(outs[1]).all()
    assert np.abs(outs[0] - outs[1]).max() <= bar * np.abs(outs[0]).max()


@pytest.mark.parametrize("d", D)
@pytest.mark.parametrize("precision", [P.H2_FP64, P.H2_MIXED], ids=["fp64", "mixed"])
def test_gmres_with_ilut_reaches_1e10(d, precision):
    """Section 5.5: GMRES to 1e-10 on the accurate H^2 matrix, preconditioned
    by the ILUt of the sparsified coarse one."""
    note(f"gmres ilut d={d} precision={precision}")
    c = case(d)
    f = P.h2_factor_S(P.h2_sparsify(c["hc"], precision), P.H2_FACTOR_ILUT, 1e-2)
    b = np.random.default_rng(7).standard_normal((N, 2))
    xs = dev(np.zeros_like(b))
    info = P.h2_solve_with(c["hf"], f, dev(b), xs, tol=1e-10, max_iter=60)
    note(f"  gmres steps {info['gmres_steps']} residual {info['residual']:.2e}")
    assert info["residual"] <= 1e-10 and 0 < info["gmres_steps"] <= 20
    a = c["fine"].dense()
    perm = c["fine"].tree.perm
    ref = from_tree(np.linalg.solve(a, b[perm]), perm)
    assert np.abs(host(xs) - ref).max() <= 1e-7 * np.abs(ref).max()


def test_ilut_option_errors():
    c = case(1e-3)
    with pytest.raises(P.H2Error) as e:
        P.h2_factor_S(P.h2_sparsify(c["hc"], P.H2_FP64), P.H2_FACTOR_ILUT, -1.0)
    assert e.value.code == P.H2_EINVAL
