"""GPU tests of the tuning table: every built tile variant of every GEMM kind
the path plans gives the same bits as the default (the tile shape changes
which wave computes an output, never the order of its sums), the Schur tile
order knob too, and the split-K knob changes results only by rounding.  The
autotuner runs end to end on a small matrix and writes a cache that loads.
"""

import json

import numpy as np
import pytest

import h2inputs
import paper_1705_04601_amd as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 4096


@pytest.fixture(autouse=True)
def _defaults():
    P.h2_tune_clear()
    yield
    P.h2_tune_clear()


def _matrix():
    x = h2inputs.points("cube", N, 41)
    return P.h2_build(x, 1.0 / (4.0 * np.pi * N), 1.0, 64, 4, 1e-8, 48)


def _rhs(nrhs, seed):
    b = h2inputs.rhs(N, nrhs, seed)
    return torch.from_numpy(np.ascontiguousarray(b.T)).cuda().T


def _apply(h, precision, b):
    f = P.h2_factor_S(P.h2_sparsify(h, precision))
    x = torch.full_like(b, float("nan"))
    P.h2_apply_inverse(f, b, x)
    torch.cuda.synchronize()
    return x.cpu().numpy()


def _used(role):
    return sorted(k for k in P.h2_tune_report()["used"] if k.startswith("gemm.") and f".{role}." in k)


def _variants(key):
    return [v for v in range(8) if _try_set(key, v)]


def _try_set(key, v):
    try:
        P.h2_tune_set(key, v)
        return True
    except P.H2Error:
        return False


@pytest.mark.parametrize("precision", [P.H2_MIXED, P.H2_FP64])
@pytest.mark.parametrize("nrhs", [96, 20])
def test_every_gemm_variant_gives_the_same_bits(precision, nrhs):
    torch.cuda.set_device(0)
    h = _matrix()
    b = _rhs(nrhs, 5)
    ref = _apply(h, precision, b)
    assert np.isfinite(ref).all()
    keys = [k for role in ("transform", "factor", "solve") for k in _used(role)]
    assert any(".solve." in k for k in keys) and any(".transform." in k for k in keys)
    checked = 0
    for key in keys:
        for v in _variants(key)[1:]:
            P.h2_tune_clear()
            P.h2_tune_set(key, v)
            got = _apply(h, precision, b)
            assert np.array_equal(got, ref), (key, v, np.abs(got - ref).max())
            checked += 1
    assert checked >= len(keys)


@pytest.mark.parametrize("nrhs", [128, 7])
def test_matvec_variants_give_the_same_bits(nrhs):
    torch.cuda.set_device(0)
    h = _matrix()
    b = _rhs(nrhs, 6)
    y0 = torch.zeros_like(b)
    P.h2_matvec(h, b, y0)
    torch.cuda.synchronize()
    keys = _used("matvec")
    assert keys
    for key in keys:
        for v in _variants(key)[1:]:
            P.h2_tune_clear()
            P.h2_tune_set(key, v)
            y = torch.zeros_like(b)
            P.h2_matvec(h, b, y)
            torch.cuda.synchronize()
            assert torch.equal(y, y0), (key, v)


def test_schur_knobs():
    torch.cuda.set_device(0)
    h = _matrix()
    b = _rhs(8, 7)
    ref = _apply(h, P.H2_MIXED, b)
    P.h2_tune_set("schur.key_z", 1)
    P.h2_tune_set("schur.order_min", 1)
    assert np.array_equal(_apply(h, P.H2_MIXED, b), ref)
    P.h2_tune_clear()
    P.h2_tune_set("schur.split_k", 16)  # splits every long target
    got = _apply(h, P.H2_MIXED, b)
    # the FP32 factor summed in another grouping: rounding only
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("precision", [P.H2_MIXED, P.H2_FP64])
def test_transposed_backward_operands_give_the_same_bits(precision):
    """The backward sweep on the transposed copy of S (K-contiguous blocks)
    against the sweep that reads S's blocks strided: the same sums in the same
    order."""
    torch.cuda.set_device(0)
    h = _matrix()
    b = _rhs(40, 12)
    P.h2_tune_set("solve.transpose", 0)
    ref = _apply(h, precision, b)
    P.h2_tune_set("solve.transpose", 1)
    got = _apply(h, precision, b)
    assert np.array_equal(got, ref)


def test_split_big_targets_gives_the_same_bits():
    """Targets of 6 to 8 blocks of 16 cut into half-edge tiles (class 0): the
    class-2 kernel no longer runs and every sum keeps its order."""
    torch.cuda.set_device(0)
    n = 8192
    x = h2inputs.points("cube", n, 43)
    h = P.h2_build(x, 1.0 / (4.0 * np.pi * n), 1.0, 128, 4, 1e-8, 64)
    bh = h2inputs.rhs(n, 8, 11)
    b = torch.from_numpy(np.ascontiguousarray(bh.T)).cuda().T

    def run():
        f = P.h2_factor_S(P.h2_sparsify(h, P.H2_MIXED))
        work = P.h2_last_work()
        xo = torch.full_like(b, float("nan"))
        P.h2_apply_inverse(f, b, xo)
        torch.cuda.synchronize()
        return xo.cpu().numpy(), work

    ref, w0 = run()
    assert w0[15] > 0  # class-2 launches at the default
    P.h2_tune_set("schur.split_big", 1)
    got, w1 = run()
    assert w1[15] == 0 and w1[11] > w0[11]
    assert np.array_equal(got, ref)


def test_autotune_writes_a_cache_that_loads(tmp_path):
    torch.cuda.set_device(0)
    h = _matrix()
    path = str(tmp_path / "tune.json")
    P.h2_autotune(h, P.H2_MIXED, 32, path)
    data = json.load(open(path))
    arch = P.h2_tune_report()["arch"]
    assert arch.startswith("gfx") and arch in data
    entries = data[arch]
    assert any(k.startswith("gemm.f32.solve.") for k in entries)
    assert "schur.split_k" in entries and "schur.key_z" in entries and "schur.split_big" in entries
    P.h2_tune_clear()
    P.h2_tune_load(path)
    for k, v in entries.items():
        assert P.h2_tune_get(k) == v
    b = _rhs(32, 9)
    x = _apply(h, P.H2_MIXED, b)
    assert np.isfinite(x).all()
    rep = P.h2_tune_report()
    assert rep["source"] == path and rep["used"]
