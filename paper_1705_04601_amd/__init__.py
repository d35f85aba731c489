"""Python binding of libh2sp (argument marshalling only).

Every function here forwards to the C ABI declared in include/h2sp.h under the
same name; all arithmetic runs in the library's HIP kernels.  Device arrays are
torch tensors on the current HIP device (torch provides memory and streams, the
library's work goes to torch's current stream).  The binding fails loudly when
the library has not been built: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libh2sp.so")
HEADER = os.path.join(HERE, "..", "include", "h2sp.h")

H2_OK, H2_EINVAL, H2_ENOMEM, H2_EDEVICE, H2_ESINGULAR, H2_ENOCONV, H2_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
H2_KERNEL_INVDIST = 0
H2_KERNEL_EXP = 1
H2_KERNEL_IFMM = 2
H2_FP64, H2_MIXED = 0, 1
H2_FACTOR_EXACT, H2_FACTOR_ILU0, H2_FACTOR_ILUT = 0, 1, 2
H2_SOLVE_AUTO, H2_SOLVE_REFINE, H2_SOLVE_GMRES = 0, 1, 2

_NAMES = {0: "H2_OK", -1: "H2_EINVAL", -2: "H2_ENOMEM", -3: "H2_EDEVICE", -4: "H2_ESINGULAR",
          -5: "H2_ENOCONV", -6: "H2_EUNSUPPORTED"}


class H2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class h2_kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("scale", ctypes.c_double), ("diag", ctypes.c_double),
                ("param", ctypes.c_double)]


class h2_build_opts(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int), ("cheb", ctypes.c_int), ("recompress_tol", ctypes.c_double),
                ("rank_cap", ctypes.c_int), ("eta", ctypes.c_double)]


class h2_sparsify_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int)]


class h2_factor_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("tau", ctypes.c_double)]


class h2_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("method", ctypes.c_int),
                ("restart", ctypes.c_int)]


class h2_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("max_rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double * 3), ("gmres_steps", ctypes.c_int),
                ("refine_steps", ctypes.c_int)]


class h2_plan_counts(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("n", "clusters", "depth", "s_blocks", "s_entries",
                                               "s_upper_entries", "q_entries", "h2_entries",
                                               "h2_close_entries", "filled_entries")] + \
               [("exact_flops", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_DP = ctypes.POINTER(ctypes.c_double)
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int32)

_SIGS = {
    "h2_last_error": (ctypes.c_char_p, []),
    "h2_set_stream": (ctypes.c_int, [_P]),
    "h2_build": (ctypes.c_int, [_DP, _I64, ctypes.c_int, ctypes.POINTER(h2_kernel),
                                ctypes.POINTER(h2_build_opts), ctypes.POINTER(_P)]),
    "h2_import": (ctypes.c_int, [_DP, _I64, ctypes.c_int, ctypes.POINTER(h2_kernel),
                                 ctypes.POINTER(h2_build_opts), _I32P, _DP, _DP, _DP, _DP,
                                 ctypes.POINTER(_P)]),
    "h2_matrix_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), _I64P, ctypes.POINTER(ctypes.c_int)]),
    "h2_matrix_export_tree": (ctypes.c_int, [_P, _I64P, _I32P]),
    "h2_matvec": (ctypes.c_int, [_P, _P, _P, _I64, _I64]),
    "h2_sparsify": (ctypes.c_int, [_P, ctypes.POINTER(h2_sparsify_opts), ctypes.POINTER(_P)]),
    "h2_sparse_info": (ctypes.c_int, [_P, _I64P, _I64P]),
    "h2_sparse_export_plan": (ctypes.c_int, [_P, _I64P, _I64P, _I64P, _I64P, _I64P, _I64P, _I64P]),
    "h2_sparse_export_block": (ctypes.c_int, [_P, _I64, _I64, _DP]),
    "h2_sparse_export_q": (ctypes.c_int, [_P, _I64, _DP]),
    "h2_factor_S": (ctypes.c_int, [_P, ctypes.POINTER(h2_factor_opts), ctypes.POINTER(_P)]),
    "h2_factor_analyze": (ctypes.c_int, [_P, _I64P, _DP]),
    "h2_plan_report": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(h2_plan_counts)]),
    "h2_tune_set": (ctypes.c_int, [ctypes.c_char_p, _I64]),
    "h2_tune_get": (ctypes.c_int, [ctypes.c_char_p, _I64P]),
    "h2_tune_clear": (ctypes.c_int, []),
    "h2_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "h2_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "h2_tune_report": (ctypes.c_int, [ctypes.c_char_p, _I64]),
    "h2_autotune": (ctypes.c_int, [_P, ctypes.c_int, _I64, ctypes.c_char_p]),
    "h2_sparsify_batch": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(h2_sparsify_opts),
                                         ctypes.POINTER(_P)]),
    "h2_factor_S_batch": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(h2_factor_opts),
                                         ctypes.POINTER(_P)]),
    "h2_solve_batch": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P),
                                      _I64P, _I64P, ctypes.POINTER(h2_solve_opts), ctypes.POINTER(h2_solve_info)]),
    "h2_solve": (ctypes.c_int, [_P, _P, _P, _I64, _I64, ctypes.POINTER(h2_solve_opts),
                                ctypes.POINTER(h2_solve_info)]),
    "h2_solve_with": (ctypes.c_int, [_P, _P, _P, _P, _I64, _I64, ctypes.POINTER(h2_solve_opts),
                                     ctypes.POINTER(h2_solve_info)]),
    "h2_apply_inverse": (ctypes.c_int, [_P, _P, _P, _I64, _I64]),
    "h2_apply_inverse_noalloc": (ctypes.c_int, [_P, _P, _P, _I64, _I64]),
    "h2_matrix_destroy": (None, [_P]),
    "h2_sparse_destroy": (None, [_P]),
    "h2_factor_destroy": (None, [_P]),
    "h2_last_timings": (ctypes.c_int, [_DP, ctypes.c_int]),
    "h2_last_work": (ctypes.c_int, [_DP, ctypes.c_int]),
}


def lib():
    """The loaded libh2sp (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def header_functions():
    """Names of the functions declared in include/h2sp.h."""
    import re
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(h2_[A-Za-z_0-9]+)\s*\(", text)))


def _check(code):
    if code != H2_OK:
        raise H2Error(code, lib().h2_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _use_torch_stream():
    """Points the library at torch's current stream (no-op without a GPU)."""
    import torch
    if torch.cuda.is_available():
        lib().h2_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


class _Handle:
    _destroy = None

    def __init__(self, ptr, keep=None):
        self.ptr = ptr
        self.keep = keep          # keeps parents alive (sparse -> matrix, factor -> sparse)

    def __del__(self):
        if self.ptr and _lib is not None:
            getattr(_lib, self._destroy)(self.ptr)
            self.ptr = None


class H2MatrixHandle(_Handle):
    _destroy = "h2_matrix_destroy"


class H2SparseHandle(_Handle):
    _destroy = "h2_sparse_destroy"


class H2FactorHandle(_Handle):
    _destroy = "h2_factor_destroy"


def _opts(leaf, cheb, tol, rank_cap, eta):
    return h2_build_opts(int(leaf), int(cheb), float(tol), int(rank_cap), float(eta))


def h2_build(points: np.ndarray, scale: float, diag: float = 1.0, leaf: int = 32, cheb: int = 4,
             tol: float = 0.0, rank_cap: int = 0, eta: float = 1.0,
             kernel: int = H2_KERNEL_INVDIST, param: float = 0.0) -> H2MatrixHandle:
    pts = np.ascontiguousarray(points, dtype=np.float64)
    _use_torch_stream()
    out = _P()
    k = h2_kernel(int(kernel), float(scale), float(diag), float(param))
    o = _opts(leaf, cheb, tol, rank_cap, eta)
    _check(lib().h2_build(_dptr(pts), pts.shape[0], pts.shape[1], ctypes.byref(k), ctypes.byref(o),
                          ctypes.byref(out)))
    return H2MatrixHandle(out.value)


def h2_import(points: np.ndarray, scale: float, diag: float, leaf: int, cheb: int, eta: float,
              rank: np.ndarray, nodes: np.ndarray, proj: np.ndarray, leaf_basis: np.ndarray,
              transfer: np.ndarray, kernel: int = H2_KERNEL_INVDIST, param: float = 0.0) -> H2MatrixHandle:
    pts = np.ascontiguousarray(points, dtype=np.float64)
    rank = np.ascontiguousarray(rank, dtype=np.int32)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (nodes, proj, leaf_basis, transfer)]
    arrs = [a if a.size else np.zeros(1) for a in arrs]
    _use_torch_stream()
    out = _P()
    k = h2_kernel(int(kernel), float(scale), float(diag), float(param))
    o = _opts(leaf, cheb, 0.0, 0, eta)
    _check(lib().h2_import(_dptr(pts), pts.shape[0], pts.shape[1], ctypes.byref(k), ctypes.byref(o),
                           rank.ctypes.data_as(_I32P), *[_dptr(a) for a in arrs], ctypes.byref(out)))
    return H2MatrixHandle(out.value)


def h2_matrix_info(h: H2MatrixHandle):
    depth, pts = ctypes.c_int(), ctypes.c_int()
    ncl = ctypes.c_int64()
    _check(lib().h2_matrix_info(h.ptr, ctypes.byref(depth), ctypes.byref(ncl), ctypes.byref(pts)))
    return depth.value, ncl.value, pts.value


def h2_matrix_export_tree(h: H2MatrixHandle, n: int):
    depth, ncl, _ = h2_matrix_info(h)
    perm = np.zeros(n, dtype=np.int64)
    rank = np.zeros(ncl, dtype=np.int32)
    _check(lib().h2_matrix_export_tree(h.ptr, perm.ctypes.data_as(_I64P), rank.ctypes.data_as(_I32P)))
    return perm, rank


def _dev(t):
    return ctypes.c_void_p(t.data_ptr())


def h2_matvec(h: H2MatrixHandle, x, y):
    """y = A_H2 x; x, y: float64 CUDA tensors (n, nrhs) column-major, i.e. x.T contiguous."""
    _use_torch_stream()
    n, nrhs, ld = _colmajor(x)
    _colmajor(y)
    _check(lib().h2_matvec(h.ptr, _dev(x), _dev(y), nrhs, ld))


def _colmajor(t):
    if t.dim() == 1:
        return t.shape[0], 1, t.shape[0]
    n, nrhs = t.shape
    if t.stride(0) != 1:
        raise ValueError("device arrays must be column-major (use t.T.contiguous().T)")
    return n, nrhs, t.stride(1) if nrhs > 1 else n


def h2_sparsify(h: H2MatrixHandle, precision: int = H2_FP64) -> H2SparseHandle:
    _use_torch_stream()
    out = _P()
    o = h2_sparsify_opts(int(precision))
    _check(lib().h2_sparsify(h.ptr, ctypes.byref(o), ctypes.byref(out)))
    return H2SparseHandle(out.value, keep=h)


def h2_sparse_info(sp: H2SparseHandle):
    b, e = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().h2_sparse_info(sp.ptr, ctypes.byref(b), ctypes.byref(e)))
    return b.value, e.value


def h2_sparse_export_plan(sp: H2SparseHandle):
    _, ncl, _ = h2_matrix_info(sp.keep)
    nb, _ = h2_sparse_info(sp)
    arr = [np.zeros(ncl, dtype=np.int64) for _ in range(5)]
    rowptr = np.zeros(ncl + 1, dtype=np.int64)
    colidx = np.zeros(max(nb, 1), dtype=np.int64)
    _check(lib().h2_sparse_export_plan(sp.ptr, *[a.ctypes.data_as(_I64P) for a in arr],
                                       rowptr.ctypes.data_as(_I64P), colidx.ctypes.data_as(_I64P)))
    return dict(n_act=arr[0], kept=arr[1], nonbasis=arr[2], soff=arr[3], elim=arr[4],
                rowptr=rowptr, colidx=colidx[:nb])


def h2_sparse_export_block(sp: H2SparseHandle, t: int, s: int, mt: int, ms: int) -> np.ndarray:
    out = np.zeros(mt * ms)
    _check(lib().h2_sparse_export_block(sp.ptr, int(t), int(s), _dptr(out)))
    return out.reshape(ms, mt).T


def h2_sparse_export_q(sp: H2SparseHandle, t: int, n: int) -> np.ndarray:
    out = np.zeros(n * n)
    _check(lib().h2_sparse_export_q(sp.ptr, int(t), _dptr(out)))
    return out.reshape(n, n).T


def h2_factor_S(sp: H2SparseHandle, mode: int = H2_FACTOR_ILU0, tau: float = 0.0) -> H2FactorHandle:
    _use_torch_stream()
    out = _P()
    o = h2_factor_opts(int(mode), float(tau))
    _check(lib().h2_factor_S(sp.ptr, ctypes.byref(o), ctypes.byref(out)))
    return H2FactorHandle(out.value, keep=sp)


def _handles(hs):
    arr = (_P * len(hs))(*[h.ptr for h in hs])
    return arr


def h2_sparsify_batch(hs, precision: int = H2_FP64):
    """Sparsifies several H^2 matrices in one level sweep; a handle per matrix."""
    _use_torch_stream()
    outs = (_P * len(hs))()
    o = h2_sparsify_opts(int(precision))
    _check(lib().h2_sparsify_batch(_handles(hs), len(hs), ctypes.byref(o), outs))
    return [H2SparseHandle(outs[i], keep=h) for i, h in enumerate(hs)]


def h2_factor_S_batch(sps, mode: int = H2_FACTOR_ILU0, tau: float = 0.0):
    _use_torch_stream()
    outs = (_P * len(sps))()
    o = h2_factor_opts(int(mode), float(tau))
    _check(lib().h2_factor_S_batch(_handles(sps), len(sps), ctypes.byref(o), outs))
    return [H2FactorHandle(outs[i], keep=sp) for i, sp in enumerate(sps)]


def h2_solve_batch(fs, bs, xs, tol: float = 1e-10, max_iter: int = 30, check: bool = True):
    """Solves every instance (b[i], x[i]: float64 CUDA tensors, column-major)."""
    _use_torch_stream()
    cnt = len(fs)
    shapes = [_colmajor(b) for b in bs]
    for x in xs:
        _colmajor(x)
    barr = (_P * cnt)(*[b.data_ptr() for b in bs])
    xarr = (_P * cnt)(*[x.data_ptr() for x in xs])
    nrhs = np.array([sh[1] for sh in shapes], dtype=np.int64)
    ld = np.array([sh[2] for sh in shapes], dtype=np.int64)
    o = h2_solve_opts(float(tol), int(max_iter), H2_SOLVE_AUTO, 0)
    infos = (h2_solve_info * cnt)()
    code = lib().h2_solve_batch(_handles(fs), cnt, barr, xarr, nrhs.ctypes.data_as(_I64P),
                                ld.ctypes.data_as(_I64P), ctypes.byref(o), infos)
    if check:
        _check(code)
    elif code not in (H2_OK, H2_ENOCONV):
        _check(code)
    return [_info_dict(i, code) for i in infos]


def h2_factor_analyze(sp: H2SparseHandle):
    """(filled entries, exact-mode Schur flops) of S's exact factorisation."""
    e = ctypes.c_int64()
    fl = ctypes.c_double()
    _check(lib().h2_factor_analyze(sp.ptr, ctypes.byref(e), ctypes.byref(fl)))
    return e.value, fl.value


def h2_plan_report(h: H2MatrixHandle, with_fill: bool = False) -> dict:
    """Host-only entry counts of the plan of h (S, U = V, the H^2 matrix)."""
    c = h2_plan_counts()
    _check(lib().h2_plan_report(h.ptr, int(with_fill), ctypes.byref(c)))
    return {f: getattr(c, f) for f, _ in h2_plan_counts._fields_}


def h2_tune_set(key: str, value: int) -> None:
    _check(lib().h2_tune_set(key.encode(), int(value)))


def h2_tune_get(key: str):
    """The table's entry for key, or None when the default applies."""
    v = ctypes.c_int64()
    code = lib().h2_tune_get(key.encode(), ctypes.byref(v))
    if code == H2_EINVAL and lib().h2_last_error().decode().startswith("no tuning entry"):
        return None
    _check(code)
    return v.value


def h2_tune_clear() -> None:
    _check(lib().h2_tune_clear())


def h2_tune_load(path=None) -> None:
    _check(lib().h2_tune_load(path.encode() if path else None))


def h2_tune_save(path=None) -> None:
    _check(lib().h2_tune_save(path.encode() if path else None))


def h2_tune_report() -> dict:
    import json
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().h2_tune_report(buf, len(buf)))
    return json.loads(buf.value.decode())


def h2_autotune(h: H2MatrixHandle, precision: int, nrhs: int, path=None) -> None:
    _use_torch_stream()
    _check(lib().h2_autotune(h.ptr, int(precision), int(nrhs), path.encode() if path else None))


def _info_dict(info, code):
    return dict(iters=info.iters, residual=info.max_rel_residual, code=code,
                t_precond=info.seconds[0], t_matvec=info.seconds[1], t_plan=info.seconds[2],
                gmres_steps=info.gmres_steps, refine_steps=info.refine_steps)


def h2_solve(f: H2FactorHandle, b, x, tol: float = 1e-10, max_iter: int = 30, check: bool = True,
             method: int = H2_SOLVE_AUTO, restart: int = 0):
    """x = A_H2^{-1} b (refinement, GMRES fallback or GMRES); b, x float64 CUDA
    tensors (n, nrhs), column-major."""
    _use_torch_stream()
    n, nrhs, ld = _colmajor(b)
    o = h2_solve_opts(float(tol), int(max_iter), int(method), int(restart))
    info = h2_solve_info()
    code = lib().h2_solve(f.ptr, _dev(b), _dev(x), nrhs, ld, ctypes.byref(o), ctypes.byref(info))
    if check or code not in (H2_OK, H2_ENOCONV):
        _check(code)
    return _info_dict(info, code)


def h2_solve_with(a: H2MatrixHandle, f: H2FactorHandle, b, x, tol: float = 1e-10, max_iter: int = 30,
                  check: bool = True, method: int = H2_SOLVE_GMRES, restart: int = 0):
    """x = A^{-1} b for the matrix `a`, with the factor `f` of another H^2
    matrix of the same points as preconditioner."""
    _use_torch_stream()
    n, nrhs, ld = _colmajor(b)
    o = h2_solve_opts(float(tol), int(max_iter), int(method), int(restart))
    info = h2_solve_info()
    code = lib().h2_solve_with(a.ptr, f.ptr, _dev(b), _dev(x), nrhs, ld, ctypes.byref(o), ctypes.byref(info))
    if check or code not in (H2_OK, H2_ENOCONV):
        _check(code)
    return _info_dict(info, code)


def h2_apply_inverse(f: H2FactorHandle, b, x):
    _use_torch_stream()
    n, nrhs, ld = _colmajor(b)
    _check(lib().h2_apply_inverse(f.ptr, _dev(b), _dev(x), nrhs, ld))


def h2_apply_inverse_noalloc(f: H2FactorHandle, b, x):
    """h2_apply_inverse with no device allocation (the library's static scratch)."""
    _use_torch_stream()
    n, nrhs, ld = _colmajor(b)
    _check(lib().h2_apply_inverse_noalloc(f.ptr, _dev(b), _dev(x), nrhs, ld))


def h2_last_timings():
    out = np.zeros(12)
    _check(lib().h2_last_timings(_dptr(out), 12))
    return out


def h2_last_work():
    out = np.zeros(20)
    _check(lib().h2_last_work(_dptr(out), 20))
    return out
