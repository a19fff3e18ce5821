"""ctypes binding of ``libpichol.so`` (C-ABI declared in include/pichol.h).

Every function here has the name and argument order of the C entry point it
calls.  Device pointers are passed as torch tensors on the current HIP
device (float64 / int32, contiguous); host arrays (lambda values, fold
sizes) as anything numpy can convert; the HIP stream is torch's current
stream unless one is given.  The functions only marshal arguments: every
step of the computation runs in the library's kernels.  There is no
fallback: when the library is missing, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PICHOL_LIB selects another build of the library (e.g. for A/B timing).
LIB_PATH = os.environ.get("PICHOL_LIB") or os.path.join(_HERE, "libpichol.so")

PICHOL_OK = 0
PICHOL_ERR_ARG = -1
PICHOL_ERR_WORKSPACE = -2
PICHOL_ERR_HIP = -3
PICHOL_ERR_NOT_PD = -4
PICHOL_ERR_DATA = -5
PICHOL_METHOD_INTERP = 1
PICHOL_METHOD_EXACT = 2
PICHOL_METHOD_GRAD = 4
PICHOL_METHOD_PINRMSE = 8
PICHOL_LAYOUT_ROWWISE = 1
PICHOL_LAYOUT_FULL = 2
PICHOL_LAYOUT_RECURSIVE = 3
PICHOL_LAYOUT_TILE = 4
PICHOL_OPT_LOOKAHEAD = 1
PICHOL_OPT_PANEL_GROUP = 2
PICHOL_OPT_SOLVE_FORM = 3
PICHOL_PREC_FP64 = 0
PICHOL_PREC_MIXED = 1
PICHOL_MAX_REFINE = 16
NB = 128

_lib = None


class PicholError(RuntimeError):
    def __init__(self, name, status, msg):
        super().__init__(f"{name} failed with status {status}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    """pichol_problem."""
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int64),
                ("c", ctypes.c_int64), ("k", ctypes.c_int32),
                ("g", ctypes.c_int32), ("r", ctypes.c_int32),
                ("q", ctypes.c_int32), ("normalize", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("basis", ctypes.c_int32),
                ("ldx", ctypes.c_int64), ("ldy", ctypes.c_int64)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_sz = ctypes.c_size_t
_pprob = ctypes.POINTER(Problem)


class BatchItem(ctypes.Structure):
    """pichol_batch_item."""
    _fields_ = [("p", Problem), ("X", _vp), ("Y", _vp), ("lam_s", _vp),
                ("lam_grid", _vp), ("lam_ref", _dbl), ("err", _vp), ("W", _vp),
                ("info", _vp), ("flags", _vp)]


class BatchTuning(ctypes.Structure):
    """pichol_batch_tuning."""
    _fields_ = [("streams", _i32), ("order", _i32), ("panel_group", _i32 * 32),
                ("solve_form", _i32 * 32)]


_pitem = ctypes.POINTER(BatchItem)
_ptune = ctypes.POINTER(BatchTuning)

_SIGNATURES = {
    "pichol_packed_elems": (_i64, [_i64]),
    "pichol_padded_order": (_i64, [_i64]),
    "pichol_slab_cols": (_i64, [_i64, _i64]),
    "pichol_pack": (_i32, [_i64, _i32, _vp, _i64, _vp, _vp]),
    "pichol_unpack": (_i32, [_i64, _i32, _vp, _vp, _i64, _vp]),
    "pichol_gram": (_i32, [_pprob, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pichol_potrf_workspace": (_sz, [_i32, _i32]),
    "pichol_potrf_shifted_batched": (_i32, [_i64, _i32, _vp, _i32, _vp, _vp,
                                            _vp, _vp, _sz, _i32, _vp]),
    "pichol_fit": (_i32, [_i64, _i32, _i32, _i32, _vp, _dbl, _vp, _vp, _vp,
                          _vp]),
    "pichol_lambda_workspace": (_sz, [_i32]),
    "pichol_factor_nrmse_workspace": (_sz, [_i64, _i32]),
    "pichol_factor_nrmse": (_i32, [_i64, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "pichol_holdout_nrmse": (_i32, [_pprob, _vp, _vp, _vp, _vp]),
    "pichol_solve_interp_workspace": (_sz, [_i64, _i32, _i32, _i32]),
    "pichol_eval": (_i32, [_i64, _i32, _i32, _vp, _i32, _vp, _dbl, _vp, _vp,
                           _sz, _vp]),
    "pichol_solve_interp": (_i32, [_i64, _i32, _i32, _i32, _vp, _vp, _vp,
                                   _i32, _vp, _dbl, _vp, _vp, _vp, _sz, _vp]),
    "pichol_solve_factors": (_i32, [_i64, _i32, _i32, _i32, _vp, _vp, _vp,
                                    _vp, _vp]),
    "pichol_holdout_workspace": (_sz, [_i64, _i32, _i32, _i32]),
    "pichol_holdout": (_i32, [_i64, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp,
                              _vp, _vp, _vp, _sz, _vp]),
    "pichol_holdout_noalloc": (_i32, [_i64, _i32, _i32, _i32, _vp, _vp, _vp,
                                      _vp, _vp, _vp, _vp, _vp]),
    "pichol_holdout_direct_workspace": (_sz, [_pprob]),
    "pichol_holdout_direct": (_i32, [_pprob, _vp, _vp, _vp, _vp, _vp, _vp, _sz,
                                     _vp]),
    "pichol_slab_to_weights": (_i32, [_i64, _i32, _i32, _i32, _vp, _vp, _vp]),
    "pichol_workspace_size": (_i32, [_pprob, _i32, ctypes.POINTER(_sz)]),
    "pichol_cv_gram": (_i32, [_pprob, _vp, _vp, _vp, _sz, _vp]),
    "pichol_cv_interp": (_i32, [_pprob, _vp, _vp, _dbl, _vp, _sz, _vp, _vp,
                                _vp, _vp, _vp]),
    "pichol_cv_exact": (_i32, [_pprob, _vp, _vp, _sz, _vp, _vp, _vp, _vp,
                               _vp]),
    "pichol_cv_interp_grad": (_i32, [_pprob, _vp, _vp, _dbl, _vp, _sz, _vp,
                                     _vp, _vp, _vp, _vp, _vp]),
    "pichol_cv_exact_grad": (_i32, [_pprob, _vp, _vp, _sz, _vp, _vp, _vp, _vp,
                                    _vp, _vp]),
    "pichol_cv_pinrmse": (_i32, [_pprob, _vp, _vp, _dbl, _vp, _sz, _vp, _vp,
                                 _vp, _vp, _vp]),
    "pichol_cv": (_i32, [_pprob, _vp, _vp, _vp, _vp, _dbl, _vp, _sz, _vp, _vp,
                         _vp, _vp, _vp]),
    "pichol_exact_cv": (_i32, [_pprob, _vp, _vp, _vp, _vp, _sz, _vp, _vp, _vp,
                               _vp, _vp]),
    "pichol_vector_length": (_i64, [_i64, _i32]),
    "pichol_vectorize": (_i32, [_i64, _i32, _vp, _i32, _i32, _vp, _vp]),
    "pichol_fit_vec": (_i32, [_i64, _i32, _i32, _i32, _vp, _dbl, _vp, _vp, _vp]),
    "pichol_eval_vec": (_i32, [_i64, _i32, _i32, _vp, _i32, _vp, _dbl, _vp, _vp,
                               _sz, _vp]),
    "pichol_batch_workspace_size": (_i32, [_i32, _pitem, _i32,
                                           ctypes.POINTER(_sz)]),
    "pichol_cv_batch": (_i32, [_i32, _pitem, _i32, _ptune, _vp, _sz, _vp]),
    "pichol_batch_buckets": (_i32, [_i32, _pitem, _i32]),
    "pichol_cv_batch_graph": (_i32, [_i32, _pitem, _i32, _ptune, _vp, _sz,
                                     ctypes.POINTER(_vp)]),
    "pichol_graph_launch": (_i32, [_vp, _vp]),
    "pichol_graph_begin": (_i32, [_vp]),
    "pichol_graph_end": (_i32, [_vp, ctypes.POINTER(_vp)]),
    "pichol_graph_destroy": (_i32, [_vp]),
    "pichol_check": (_i32, [_vp, _i64, _vp, _i64, _vp]),
    "pichol_set_option": (_i32, [_i32, _i32]),
    "pichol_get_option": (_i32, [_i32]),
    "pichol_profile_start": (_i32, [_i32]),
    "pichol_profile_stop": (_i32, []),
    "pichol_profile_summary": (_i32, [_i32, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(_i64),
                                      ctypes.POINTER(_dbl)]),
    "pichol_profile_reset": (_i32, []),
    "pichol_status_string": (ctypes.c_char_p, [_i32]),
    "pichol_last_error": (ctypes.c_char_p, []),
}

EXPORTED = tuple(_SIGNATURES)


def load(path: str | None = None):
    """Load the HIP library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_1404_0466_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(name, status):
    if status != PICHOL_OK:
        lib = load()
        msg = lib.pichol_status_string(status).decode()
        extra = lib.pichol_last_error().decode()
        raise PicholError(name, status, msg + (f" ({extra})" if extra else ""))


def _dev(t, dtype=None):
    """Device pointer of a contiguous tensor (None passes NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a HIP device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


class _Host:
    """Keeps a host array alive for the duration of a call."""

    def __init__(self, a, dtype):
        self.arr = np.ascontiguousarray(np.asarray(a, dtype=dtype))
        self.ptr = ctypes.c_void_p(self.arr.ctypes.data)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _f64():
    import torch
    return torch.float64


def _i32t():
    import torch
    return torch.int32


# ------------------------------------------------------------------ layout

def pichol_packed_elems(d: int) -> int:
    return int(load().pichol_packed_elems(d))


def pichol_padded_order(d: int) -> int:
    return int(load().pichol_padded_order(d))


def pichol_slab_cols(q: int, c: int) -> int:
    return int(load().pichol_slab_cols(q, c))


def pichol_pack(d, nmat, A, lda, P, stream=None):
    _check("pichol_pack", load().pichol_pack(d, nmat, _dev(A, _f64()), lda,
                                             _dev(P, _f64()), _stream(stream)))


def pichol_unpack(d, nmat, P, A, lda, stream=None):
    _check("pichol_unpack", load().pichol_unpack(d, nmat, _dev(P, _f64()),
                                                 _dev(A, _f64()), lda,
                                                 _stream(stream)))


# ------------------------------------------------------------------ steps

def make_problem(n, d, c, k, g=1, r=0, q=1, normalize=True, ldx=None,
                 ldy=None, precision=PICHOL_PREC_FP64, refine=0,
                 basis=0) -> Problem:
    return Problem(n, d, c, k, g, r, q, int(bool(normalize)), int(precision),
                   int(refine), int(basis), d if ldx is None else ldx,
                   c if ldy is None else ldy)


def pichol_gram(p: Problem, X, Y, G, C, yy, H, B, stream=None):
    _check("pichol_gram", load().pichol_gram(
        ctypes.byref(p), _dev(X, _f64()), _dev(Y, _f64()), _dev(G, _f64()),
        _dev(C, _f64()), _dev(yy, _f64()), _dev(H, _f64()), _dev(B, _f64()),
        _stream(stream)))


def pichol_potrf_workspace(nmat: int, nshift: int) -> int:
    return int(load().pichol_potrf_workspace(nmat, nshift))


def pichol_potrf_shifted_batched(d, nmat, H, nshift, lam, L, info, ws,
                                 ws_bytes, precision=PICHOL_PREC_FP64,
                                 stream=None):
    lam_h = _Host(lam, np.float64)
    _check("pichol_potrf_shifted_batched", load().pichol_potrf_shifted_batched(
        d, nmat, _dev(H, _f64()), nshift, lam_h.ptr, _dev(L, _f64()),
        _dev(info, _i32t()), _dev(ws), ws_bytes, int(precision),
        _stream(stream)))


def pichol_fit(d, nmat, g, r, lam_s, lam_ref, L, theta, theta_t, stream=None):
    lam_h = _Host(lam_s, np.float64)
    _check("pichol_fit", load().pichol_fit(
        d, nmat, g, r, lam_h.ptr, float(lam_ref), _dev(L, _f64()),
        _dev(theta, _f64()), _dev(theta_t, _f64()), _stream(stream)))


def pichol_lambda_workspace(nlam: int) -> int:
    return int(load().pichol_lambda_workspace(nlam))


def pichol_solve_interp_workspace(d: int, nmat: int, q: int, c: int) -> int:
    return int(load().pichol_solve_interp_workspace(d, nmat, q, c))


def pichol_factor_nrmse_workspace(d: int, nmat: int) -> int:
    return int(load().pichol_factor_nrmse_workspace(d, nmat))


def pichol_factor_nrmse(d, nmat, Lhat, L, out, ws, ws_bytes, stream=None):
    _check("pichol_factor_nrmse", load().pichol_factor_nrmse(
        d, nmat, _dev(Lhat, _f64()), _dev(L, _f64()), _dev(out, _f64()),
        _dev(ws), ws_bytes, _stream(stream)))


def pichol_holdout_nrmse(p: Problem, Y, err, nrmse, stream=None):
    _check("pichol_holdout_nrmse", load().pichol_holdout_nrmse(
        ctypes.byref(p), _dev(Y, _f64()), _dev(err, _f64()), _dev(nrmse, _f64()),
        _stream(stream)))


def pichol_eval(d, nmat, r, theta, nlam, lam, lam_ref, Lhat, ws, ws_bytes,
                stream=None):
    lam_h = _Host(lam, np.float64)
    _check("pichol_eval", load().pichol_eval(
        d, nmat, r, _dev(theta, _f64()), nlam, lam_h.ptr, float(lam_ref),
        _dev(Lhat, _f64()), _dev(ws), ws_bytes, _stream(stream)))


def pichol_solve_interp(d, nmat, c, r, theta, theta_t, B, q, lam, lam_ref, Z,
                        flags, ws, ws_bytes, stream=None):
    lam_h = _Host(lam, np.float64)
    _check("pichol_solve_interp", load().pichol_solve_interp(
        d, nmat, c, r, _dev(theta, _f64()), _dev(theta_t, _f64()),
        _dev(B, _f64()), q, lam_h.ptr, float(lam_ref), _dev(Z, _f64()),
        _dev(flags, _i32t()), _dev(ws), ws_bytes, _stream(stream)))


def pichol_solve_factors(d, nmat, nper, c, L, B, Z, flags, stream=None):
    _check("pichol_solve_factors", load().pichol_solve_factors(
        d, nmat, nper, c, _dev(L, _f64()), _dev(B, _f64()), _dev(Z, _f64()),
        _dev(flags, _i32t()), _stream(stream)))


def pichol_holdout_workspace(d, nmat, q, c) -> int:
    return int(load().pichol_holdout_workspace(d, nmat, q, c))


def pichol_holdout(d, nmat, c, q, Z, G, C, yy, nv, err, flags, ws, ws_bytes,
                   stream=None):
    nv_h = _Host(nv, np.int64)
    _check("pichol_holdout", load().pichol_holdout(
        d, nmat, c, q, _dev(Z, _f64()), _dev(G, _f64()), _dev(C, _f64()),
        _dev(yy, _f64()), nv_h.ptr, _dev(err, _f64()), _dev(flags, _i32t()),
        _dev(ws), ws_bytes, _stream(stream)))


PICHOL_HOLDOUT_SCRATCH_BYTES = 16 << 20


def pichol_holdout_noalloc(d, nmat, c, q, Z, G, C, yy, nv, err, flags,
                           stream=None):
    nv_h = _Host(nv, np.int64)
    _check("pichol_holdout_noalloc", load().pichol_holdout_noalloc(
        d, nmat, c, q, _dev(Z, _f64()), _dev(G, _f64()), _dev(C, _f64()),
        _dev(yy, _f64()), nv_h.ptr, _dev(err, _f64()), _dev(flags, _i32t()),
        _stream(stream)))


def pichol_holdout_direct_workspace(p: Problem) -> int:
    return int(load().pichol_holdout_direct_workspace(ctypes.byref(p)))


def pichol_holdout_direct(p: Problem, X, Y, Z, err, flags, ws, ws_bytes,
                          stream=None):
    _check("pichol_holdout_direct", load().pichol_holdout_direct(
        ctypes.byref(p), _dev(X, _f64()), _dev(Y, _f64()), _dev(Z, _f64()),
        _dev(err, _f64()), _dev(flags, _i32t()), _dev(ws), ws_bytes,
        _stream(stream)))


def pichol_slab_to_weights(d, nmat, q, c, Z, W, stream=None):
    _check("pichol_slab_to_weights", load().pichol_slab_to_weights(
        d, nmat, q, c, _dev(Z, _f64()), _dev(W, _f64()), _stream(stream)))


# ------------------------------------------------------------------ pipelines

def pichol_workspace_size(p: Problem, methods: int) -> int:
    out = _sz(0)
    _check("pichol_workspace_size", load().pichol_workspace_size(
        ctypes.byref(p), methods, ctypes.byref(out)))
    return int(out.value)


def pichol_cv_gram(p: Problem, X, Y, ws, ws_bytes, stream=None):
    _check("pichol_cv_gram", load().pichol_cv_gram(
        ctypes.byref(p), _dev(X, _f64()), _dev(Y, _f64()), _dev(ws), ws_bytes,
        _stream(stream)))


def pichol_cv_interp(p: Problem, lam_s, lam_grid, lam_ref, ws, ws_bytes, err,
                     W, info, flags, stream=None):
    ls = _Host(lam_s, np.float64)
    lg = _Host(lam_grid, np.float64)
    _check("pichol_cv_interp", load().pichol_cv_interp(
        ctypes.byref(p), ls.ptr, lg.ptr, float(lam_ref), _dev(ws), ws_bytes,
        _dev(err, _f64()), _dev(W, _f64()), _dev(info, _i32t()),
        _dev(flags, _i32t()), _stream(stream)))


def pichol_cv_exact(p: Problem, lam_grid, ws, ws_bytes, err, W, info, flags,
                    stream=None):
    lg = _Host(lam_grid, np.float64)
    _check("pichol_cv_exact", load().pichol_cv_exact(
        ctypes.byref(p), lg.ptr, _dev(ws), ws_bytes, _dev(err, _f64()),
        _dev(W, _f64()), _dev(info, _i32t()), _dev(flags, _i32t()),
        _stream(stream)))


def pichol_cv_interp_grad(p: Problem, lam_s, lam_grid, lam_ref, ws, ws_bytes, err,
                          dlog, W, info, flags, stream=None):
    ls = _Host(lam_s, np.float64)
    lg = _Host(lam_grid, np.float64)
    _check("pichol_cv_interp_grad", load().pichol_cv_interp_grad(
        ctypes.byref(p), ls.ptr, lg.ptr, float(lam_ref), _dev(ws), ws_bytes,
        _dev(err, _f64()), _dev(dlog, _f64()), _dev(W, _f64()),
        _dev(info, _i32t()), _dev(flags, _i32t()), _stream(stream)))


def pichol_cv_exact_grad(p: Problem, lam_grid, ws, ws_bytes, err, dlog, W, info,
                         flags, stream=None):
    lg = _Host(lam_grid, np.float64)
    _check("pichol_cv_exact_grad", load().pichol_cv_exact_grad(
        ctypes.byref(p), lg.ptr, _dev(ws), ws_bytes, _dev(err, _f64()),
        _dev(dlog, _f64()), _dev(W, _f64()), _dev(info, _i32t()),
        _dev(flags, _i32t()), _stream(stream)))


def pichol_cv_pinrmse(p: Problem, lam_s, lam_grid, lam_ref, ws, ws_bytes, err,
                      err_s, info, flags, stream=None):
    ls = _Host(lam_s, np.float64)
    lg = _Host(lam_grid, np.float64)
    _check("pichol_cv_pinrmse", load().pichol_cv_pinrmse(
        ctypes.byref(p), ls.ptr, lg.ptr, float(lam_ref), _dev(ws), ws_bytes,
        _dev(err, _f64()), _dev(err_s, _f64()), _dev(info, _i32t()),
        _dev(flags, _i32t()), _stream(stream)))


def pichol_cv(p: Problem, X, Y, lam_s, lam_grid, lam_ref, ws, ws_bytes, err, W,
              info, flags, stream=None):
    ls = _Host(lam_s, np.float64)
    lg = _Host(lam_grid, np.float64)
    _check("pichol_cv", load().pichol_cv(
        ctypes.byref(p), _dev(X, _f64()), _dev(Y, _f64()), ls.ptr, lg.ptr,
        float(lam_ref), _dev(ws), ws_bytes, _dev(err, _f64()), _dev(W, _f64()),
        _dev(info, _i32t()), _dev(flags, _i32t()), _stream(stream)))


def pichol_exact_cv(p: Problem, X, Y, lam_grid, ws, ws_bytes, err, W, info,
                    flags, stream=None):
    lg = _Host(lam_grid, np.float64)
    _check("pichol_exact_cv", load().pichol_exact_cv(
        ctypes.byref(p), _dev(X, _f64()), _dev(Y, _f64()), lg.ptr, _dev(ws),
        ws_bytes, _dev(err, _f64()), _dev(W, _f64()), _dev(info, _i32t()),
        _dev(flags, _i32t()), _stream(stream)))


def pichol_check(info, n_info, flags, n_flags, stream=None) -> int:
    """Returns the status code (does not raise on NOT_PD / DATA)."""
    return int(load().pichol_check(_dev(info, _i32t()), n_info,
                                   _dev(flags, _i32t()), n_flags,
                                   _stream(stream)))


# ------------------------------------------------------------------ options

def pichol_set_option(option: int, value: int):
    _check("pichol_set_option", load().pichol_set_option(option, value))


def pichol_get_option(option: int) -> int:
    return int(load().pichol_get_option(option))


# ------------------------------------------------------------------ profiling

def pichol_profile_start(capacity: int):
    _check("pichol_profile_start", load().pichol_profile_start(capacity))


def pichol_profile_stop():
    _check("pichol_profile_stop", load().pichol_profile_stop())


def pichol_profile_summary(max_kernels: int = 256) -> dict:
    """{kernel name: (launches, total milliseconds)} of the recorded
    launches."""
    names = (ctypes.c_char_p * max_kernels)()
    launches = (_i64 * max_kernels)()
    total = (_dbl * max_kernels)()
    n = load().pichol_profile_summary(max_kernels, names, launches, total)
    if n < 0:
        raise PicholError("pichol_profile_summary", PICHOL_ERR_HIP,
                          load().pichol_last_error().decode())
    return {names[i].decode(): (int(launches[i]), float(total[i]))
            for i in range(min(n, max_kernels))}


def pichol_profile_reset():
    _check("pichol_profile_reset", load().pichol_profile_reset())


# ------------------------------------------------------------------ layouts

def pichol_vector_length(d: int, layout: int) -> int:
    return int(load().pichol_vector_length(d, layout))


def pichol_vectorize(d, nmat, L, layout, h0, T, stream=None):
    _check("pichol_vectorize", load().pichol_vectorize(
        d, nmat, _dev(L, _f64()), layout, h0, _dev(T, _f64()), _stream(stream)))


def pichol_fit_vec(N, nmat, g, r, lam_s, lam_ref, T, theta, stream=None):
    ls = _Host(lam_s, np.float64)
    _check("pichol_fit_vec", load().pichol_fit_vec(
        N, nmat, g, r, ls.ptr, float(lam_ref), _dev(T, _f64()), _dev(theta, _f64()),
        _stream(stream)))


def pichol_eval_vec(N, nmat, r, theta, nlam, lam, lam_ref, out, ws, ws_bytes,
                    stream=None):
    lh = _Host(lam, np.float64)
    _check("pichol_eval_vec", load().pichol_eval_vec(
        N, nmat, r, _dev(theta, _f64()), nlam, lh.ptr, float(lam_ref),
        _dev(out, _f64()), _dev(ws), ws_bytes, _stream(stream)))


# ------------------------------------------------------------------ batching

def _ptr(t, dtype=None):
    """Device pointer of a tensor, or an integer address passed through (for
    host-only calls such as the workspace size), or NULL for None."""
    if t is None or isinstance(t, int):
        return t
    return _dev(t, dtype)


class Batch:
    """A ctypes array of pichol_batch_item built from dicts with the keys
    p (Problem), X, Y, err, W, info, flags (device tensors, W may be None),
    lam_s (host, interpolated method), lam_grid (host), lam_ref.  Keeps the
    host lambda arrays alive as long as the batch object lives."""

    def __init__(self, entries):
        self.n = len(entries)
        self.items = (BatchItem * max(1, self.n))()
        self._keep = []
        for i, e in enumerate(entries):
            ls = _Host(e["lam_s"], np.float64) if e.get("lam_s") is not None else None
            lg = _Host(e["lam_grid"], np.float64)
            self._keep += [ls, lg]
            it = self.items[i]
            it.p = e["p"]
            it.X = _ptr(e["X"], _f64() if not isinstance(e["X"], int) else None)
            it.Y = _ptr(e["Y"], _f64() if not isinstance(e["Y"], int) else None)
            it.lam_s = ls.ptr if ls is not None else None
            it.lam_grid = lg.ptr
            it.lam_ref = float(e.get("lam_ref", 0.0))
            for name in ("err", "W"):
                v = e.get(name)
                setattr(it, name, _ptr(v, _f64() if v is not None and not isinstance(v, int) else None))
            for name in ("info", "flags"):
                v = e.get(name)
                setattr(it, name, _ptr(v, _i32t() if v is not None and not isinstance(v, int) else None))


def _tune(tune):
    if tune is None:
        return None
    if isinstance(tune, BatchTuning):
        return ctypes.byref(tune)
    t = BatchTuning(int(tune.get("streams", 0)), int(tune.get("order", 0)))
    for nt, gsz in (tune.get("panel_group") or {}).items():
        t.panel_group[int(nt) - 1] = int(gsz)
    for nt, form in (tune.get("solve_form") or {}).items():
        t.solve_form[int(nt) - 1] = int(form)
    return ctypes.byref(t)


def pichol_batch_workspace_size(batch: Batch, method: int) -> int:
    out = _sz(0)
    _check("pichol_batch_workspace_size", load().pichol_batch_workspace_size(
        batch.n, batch.items, method, ctypes.byref(out)))
    return int(out.value)


def pichol_batch_buckets(batch: Batch, method: int) -> int:
    return int(load().pichol_batch_buckets(batch.n, batch.items, method))


def pichol_cv_batch(batch: Batch, method: int, tune, ws, ws_bytes, stream=None):
    _check("pichol_cv_batch", load().pichol_cv_batch(
        batch.n, batch.items, method, _tune(tune), _dev(ws), ws_bytes,
        _stream(stream)))


def pichol_cv_batch_graph(batch: Batch, method: int, tune, ws, ws_bytes):
    """Returns the graph handle (pass it to pichol_graph_launch / _destroy)."""
    g = _vp(None)
    _check("pichol_cv_batch_graph", load().pichol_cv_batch_graph(
        batch.n, batch.items, method, _tune(tune), _dev(ws), ws_bytes,
        ctypes.byref(g)))
    return g


def pichol_graph_begin(stream=None):
    _check("pichol_graph_begin", load().pichol_graph_begin(_stream(stream)))


def pichol_graph_end(stream=None):
    g = _vp(None)
    _check("pichol_graph_end", load().pichol_graph_end(_stream(stream), ctypes.byref(g)))
    return g


def pichol_graph_launch(graph, stream=None):
    _check("pichol_graph_launch", load().pichol_graph_launch(graph, _stream(stream)))


def pichol_graph_destroy(graph):
    _check("pichol_graph_destroy", load().pichol_graph_destroy(graph))

