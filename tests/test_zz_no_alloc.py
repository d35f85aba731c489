"""GPU test of h2_apply_inverse_noalloc, the entry point that allocates no
device memory (its vectors and work lists live in the library's static
scratch array), through the C ABI.

It runs the same kernels in the same order as h2_apply_inverse, so the bar is
bit-for-bit equality with that entry point's output.  Two calls in a row, the
second with fewer right-hand sides, in both precisions; then a request too
large for the array, which must come back as EINVAL with a message, and a
call after it that still works.
"""

import ctypes

import numpy as np
import pytest

import h2inputs
import paper_1705_04601_amd as P

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev_rhs(n, nrhs, seed):
    b = h2inputs.rhs(n, nrhs, seed)
    return torch.from_numpy(np.ascontiguousarray(b.T)).cuda().T


def raw_apply(name, f, b, x):
    fn = getattr(P.lib(), name)
    n, nrhs = b.shape
    rc = fn(ctypes.c_void_p(f.ptr), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
            ctypes.c_int64(nrhs), ctypes.c_int64(b.stride(1)))
    torch.cuda.synchronize()
    return rc


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_apply_inverse(precision):
    torch.cuda.set_device(0)
    n = 3000
    x = h2inputs.points("cube", n, 31)
    sc = 1.0 / (4.0 * np.pi * n)
    h = P.h2_build(x, sc, 1.0, 32, 3, 1e-8, 27)
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_FP64 if precision == "fp64" else P.H2_MIXED))
    for call, nrhs in enumerate((16, 3)):
        b = dev_rhs(n, nrhs, 100 + call)
        ref = torch.full_like(b, float("nan"))
        out = torch.full_like(b, float("nan"))
        assert raw_apply("h2_apply_inverse", f, b, ref) == 0, P.lib().h2_last_error()
        assert raw_apply("h2_apply_inverse_noalloc", f, b, out) == 0, P.lib().h2_last_error()
        r, o = ref.cpu().numpy(), out.cpu().numpy()
        assert np.isfinite(o).all()
        assert np.array_equal(r, o), (call, np.abs(r - o).max())


def test_noalloc_rejects_requests_beyond_the_array():
    torch.cuda.set_device(0)
    n = 8192
    x = h2inputs.points("cube", n, 32)
    sc = 1.0 / (4.0 * np.pi * n)
    h = P.h2_build(x, sc, 1.0, 64, 3, 1e-8, 27)
    f = P.h2_factor_S(P.h2_sparsify(h, P.H2_MIXED))
    big = dev_rhs(n, 512, 7)  # about 4 n nrhs doubles: far above 64 MiB
    out = torch.zeros_like(big)
    rc = raw_apply("h2_apply_inverse_noalloc", f, big, out)
    assert rc == P.H2_EINVAL
    assert b"scratch" in P.lib().h2_last_error()
    assert float(out.abs().max()) == 0.0  # nothing was written
    small = dev_rhs(n, 2, 8)
    ref = torch.zeros_like(small)
    got = torch.zeros_like(small)
    assert raw_apply("h2_apply_inverse", f, small, ref) == 0
    assert raw_apply("h2_apply_inverse_noalloc", f, small, got) == 0
    assert torch.equal(ref, got)
