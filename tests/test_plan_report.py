"""CPU checks of the host-only plan report (storage counts of Sections
5.1-5.2): the counts of S, U = V and the H^2 matrix that the library plans
without device work equal those of the oracle's sparsification, and the exact
mode's fill equals the oracle's graph elimination (Sections 5.3-5.4)."""

import numpy as np
import pytest

import paper_1705_04601_amd as P
import oracle
from h2test_util import make_case


def _oracle_counts(h2, sp):
    tr = h2.tree
    m = sp.nonbasis
    s_ent = sum(int(m[t]) * int(m[s]) for (t, s) in sp.s_blocks if m[t] > 0 and m[s] > 0)
    pos = {int(c): i for i, c in enumerate(sp.order)}
    upper = [(t, s) for (t, s) in sp.s_blocks if m[t] > 0 and m[s] > 0 and pos[t] <= pos[s]]
    q_ent = sum(int(q.shape[0]) ** 2 for q in sp.q.values())
    h2e = sum(b.size for b in h2.leaf_basis.values()) + sum(t.size for t in h2.transfer.values())
    h2e += sum(int(h2.rank[t]) * int(h2.rank[s]) for k in range(tr.depth + 1) for (t, s) in h2.bt.far[k])
    close = sum(int(tr.size[t]) * int(tr.size[s]) for (t, s) in h2.bt.near[0])
    order = oracle.elimination_order(sp)
    fill = oracle.block_fill(sp, order)
    fpos = {int(c): i for i, c in enumerate(order)}
    filled = sum(int(m[t]) * int(m[s]) for (t, s) in fill if fpos[t] <= fpos[s])
    return dict(s_blocks=len(upper), s_entries=s_ent, q_entries=q_ent, h2_entries=h2e + close,
                h2_close_entries=close, filled_entries=filled)


@pytest.mark.parametrize("kind,n,seed,leaf,cheb,tol,cap,eta", [
    ("cube", 1500, 31, 32, 3, 1e-8, 27, 1.0),
    ("square", 1024, 1, 32, 4, 0.0, 16, 1.0),
    ("sphere", 2048, 12, 64, 3, 1e-6, 27, 1.0),
])
def test_plan_report_matches_oracle(kind, n, seed, leaf, cheb, tol, cap, eta):
    x, sc, h2 = make_case(kind, n, seed, leaf, cheb, tol, cap, eta)
    sp = oracle.sparsify(h2)
    want = _oracle_counts(h2, sp)
    h = P.h2_build(x, sc, 1.0, leaf, cheb, tol, cap, eta)
    got = P.h2_plan_report(h, with_fill=True)
    assert got["n"] == n and got["clusters"] == h2.tree.ncl and got["depth"] == h2.tree.depth
    for key, v in want.items():
        assert got[key] == v, (key, got[key], v)
    diag = sum(int(m) ** 2 for m in sp.nonbasis)
    assert got["s_upper_entries"] == (got["s_entries"] + diag) // 2
    # S is square of order n: the nonbasis sizes add up to n (Proposition 2.1)
    assert int(sp.nonbasis.sum()) == n
    assert got["exact_flops"] > 0


def test_plan_report_without_fill():
    x, sc, h2 = make_case("cube", 1200, 5, 32, 3, 1e-8, 27, 1.0)
    h = P.h2_build(x, sc, 1.0, 32, 3, 1e-8, 27, 1.0)
    got = P.h2_plan_report(h)
    assert got["filled_entries"] == -1 and got["exact_flops"] == -1
    assert 0 < got["s_upper_entries"] <= got["s_entries"] < 1200 * 1200


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("core", ["inv", "exp"])
def test_report_settings_reach_the_papers_accuracy(dim, core):
    """The H^2 settings of the storage report give products with random
    vectors within 1e-6 of the dense matrix of Example 5.1 or 5.2 (the accuracy
    Sections 5.1-5.2 state), at N = 4096 against the matrix written out."""
    import h2inputs
    from paper_1705_04601_amd import report
    st = report.SETTINGS[dim]
    n = 4096
    x = h2inputs.points("square" if dim == 2 else "cube", n, 11)
    if core == "exp":
        h2 = oracle.build_h2(x, st["leaf"], st["cheb"], 1.0, 3.0, st["tol"], 0, st["eta"], oracle.EXP)
    else:
        h2 = oracle.build_h2(x, st["leaf"], st["cheb"], 1.0, 0.0, st["tol"], 0, st["eta"])
    assert h2.rank.max() > 0  # some blocks are compressed
    xt = h2.x_tree
    d2 = ((xt[:, None, :] - xt[None, :, :]) ** 2).sum(-1)
    if core == "exp":
        a = 2.0 * np.eye(n) + np.exp(-d2)
    else:
        np.fill_diagonal(d2, 1.0)
        a = 1.0 / np.sqrt(d2)
        np.fill_diagonal(a, 0.0)
    v = np.random.default_rng(5).standard_normal((n, 4))
    err = np.linalg.norm(h2.matvec(v) - a @ v) / np.linalg.norm(a @ v)
    assert err < 1e-6, err
