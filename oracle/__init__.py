"""Plain FP64 CPU oracle for piCholesky cross-validation.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code with the GPU library and imports nothing from it.

The arithmetic lives in ``pichol_oracle.c`` (plain loops, FP64,
``-ffp-contract=off``); this module only builds that file with gcc, loads it
with ctypes and marshals numpy arrays.  The few helpers written here in
Python are the cross-validation bookkeeping of the paper's experiments
(fold means, argmin, gap metrics: Sec. 6.4-6.5) and the choice of the lambda
scale.

Every function works on host numpy arrays; inputs are converted to
C-contiguous float64 copies, outputs are freshly allocated.

Parity status: every entry point is pinned by the CPU tests in
``tests/test_oracle_pins.py`` (closed forms, LAPACK, SVD ridge form,
polynomial reproduction, interpolation of the samples, and the Sec. 4 main
result at tiny sizes: the degree-2 factor's error falls as the cube of the
sample width, and it stays within the theorem's bound with the constants
M_s, E_s and R evaluated as the paper writes them.  That derivation takes
vec(Gamma^T) = vec(Gamma) for a lower triangular Gamma, so its M_s^-1 v_I is
not the factor's derivative; the bound is used as printed and is loose).
The whole interpolated pipeline off the samples is pinned at small d against
the same steps composed from library routines (LAPACK Cholesky, numpy
polyfit/polyval, LAPACK triangular solves, the validation residual) and
against the same mathematics in 50-digit arithmetic.  At large d the curve
has no pin beyond these: its parity there is "parity unpinned" beyond the
oracle itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pichol_oracle.c")
_HDR = os.path.join(_HERE, "pichol_oracle.h")
_LIB = os.path.join(_HERE, "libpichol_oracle.so")
_lock = threading.Lock()
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, no FP contraction).  Returns the
    path of the shared library."""
    with _lock:
        fresh = (os.path.exists(_LIB)
                 and os.path.getmtime(_LIB) >= max(os.path.getmtime(_SRC),
                                                   os.path.getmtime(_HDR)))
        if force or not fresh:
            tmp = _LIB + ".tmp%d" % os.getpid()
            cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                   "-fno-fast-math", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    sig = {
        "orc_fold_bounds": (None, [_i64, _i32, _pi64]),
        "orc_fold_gram": (_i64, [_i64, _i64, _i64, _i32, _i32, _pd, _pd,
                                 ctypes.c_int, _pd, _pd]),
        "orc_cholesky": (_i32, [_i64, _pd, _dbl, _pd]),
        "orc_pack_lower": (None, [_i64, _pd, _pd]),
        "orc_unpack_lower": (None, [_i64, _pd, _pd]),
        "orc_fit": (_i32, [_i64, _i32, _i32, _pd, _dbl, _pd, _pd, _i32]),
        "orc_eval": (None, [_i64, _i32, _pd, _dbl, _dbl, _pd, _i32]),
        "orc_solve": (_i32, [_i64, _i64, _pd, _pd, _pd]),
        "orc_holdout_sse": (_dbl, [_i64, _i64, _i64, _pd, _i64, _pd, _i64,
                                   _pd]),
        "orc_holdout_sst": (_dbl, [_i64, _i64, _pd, _i64]),
        "orc_factor_nrmse": (_dbl, [_i64, _pd, _pd]),
        "orc_refine": (_i32, [_i64, _i64, _pd, _dbl, _pd, _pd, _pd, _i32]),
        "orc_eval_deriv": (None, [_i64, _i32, _pd, _dbl, _dbl, _pd, _i32]),
        "orc_cv_grad": (_i32, [_i64, _i64, _i64, _i32, _i32, _i32, _i32,
                               ctypes.c_int, ctypes.c_int, _pd, _pd, _pd, _pd,
                               _dbl, _pd, _pd, _pi32, _pi32, _i32]),
        "orc_cv_exact": (_i32, [_i64, _i64, _i64, _i32, _i32, ctypes.c_int,
                                _pd, _pd, _pd, _pd, _pd, _pd, _pi32, _pi32,
                                _i32]),
        "orc_cv_interp": (_i32, [_i64, _i64, _i64, _i32, _i32, _i32, _i32,
                                 ctypes.c_int, _pd, _pd, _pd, _pd, _dbl, _pd,
                                 _pd, _pd, _pd, _pi32, _pi32, _i32, _i32]),
        "orc_fold_interp": (_i32, [_i64, _i64, _i32, _i32, _i32, _pd, _pd,
                                   _i64, _pd, _i64, _pd, _i64, _pd, _pd, _dbl,
                                   _pd, _pd, _pi32, _pi32, _i32, _i32]),
        "orc_num_threads": (_i32, []),
        "orc_set_num_threads": (None, [_i32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    if a is None:
        return None
    if a.dtype == np.float64:
        return a.ctypes.data_as(_pd)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_pi32)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_pi64)
    raise TypeError(a.dtype)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (n >= 1)."""
    _load().orc_set_num_threads(int(n))


# ---------------------------------------------------------------- building blocks

def fold_bounds(n: int, k: int) -> np.ndarray:
    """Row offsets of k contiguous folds, sizes as numpy.array_split."""
    out = np.zeros(k + 1, dtype=np.int64)
    _load().orc_fold_bounds(n, k, _p(out))
    return out


def fold_gram(X, Y, k: int, f: int, normalize: bool = True):
    """H_f = X_tr^T X_tr and B_f = X_tr^T Y_tr of training fold f (Sec. 3.1),
    divided by n_tr when normalize.  Returns (H, B, n_tr)."""
    X = _f64(X)
    Y = _f64(Y)
    if Y.ndim == 1:
        Y = Y[:, None].copy()
    n, d = X.shape
    c = Y.shape[1]
    H = np.zeros((d, d))
    B = np.zeros((d, c))
    ntr = _load().orc_fold_gram(n, d, c, k, f, _p(X), _p(Y), int(normalize),
                                _p(H), _p(B))
    return H, B, int(ntr)


def cholesky(A, lam: float = 0.0):
    """Lower factor of A + lam I (Sec. 3.2) and its LAPACK-style info."""
    A = _f64(A)
    d = A.shape[0]
    L = np.zeros((d, d))
    info = _load().orc_cholesky(d, _p(A), float(lam), _p(L))
    return L, int(info)


def pack_lower(L) -> np.ndarray:
    L = _f64(L)
    d = L.shape[0]
    t = np.zeros(d * (d + 1) // 2)
    _load().orc_pack_lower(d, _p(L), _p(t))
    return t


def unpack_lower(t, d: int) -> np.ndarray:
    t = _f64(t)
    L = np.zeros((d, d))
    _load().orc_unpack_lower(d, _p(t), _p(L))
    return L


def fit(T, lam_s, r: int, lam_ref: float, basis: int = 0) -> np.ndarray:
    """Algorithm 1 steps 3-6: Theta ((r+1) x D) from the g x D targets T
    (basis 0: polynomials in lam/lam_ref; 1: in log(lam/lam_ref))."""
    T = _f64(T)
    lam_s = _f64(lam_s)
    g, D = T.shape
    Theta = np.zeros((r + 1, D))
    rc = _load().orc_fit(D, g, r, _p(lam_s), float(lam_ref), _p(T), _p(Theta),
                         int(basis))
    if rc != 0:
        raise ValueError("oracle fit rejected its arguments (r >= g, "
                         "lam_ref <= 0 or repeated samples)")
    return Theta


def evaluate(Theta, lam: float, lam_ref: float, basis: int = 0) -> np.ndarray:
    """The D fitted polynomials at lam (Sec. 3.3), as a packed vector."""
    Theta = _f64(Theta)
    r = Theta.shape[0] - 1
    D = Theta.shape[1]
    out = np.zeros(D)
    _load().orc_eval(D, r, _p(Theta), float(lam), float(lam_ref), _p(out), int(basis))
    return out


def solve(L, B):
    """Forward then back substitution with lower L (Sec. 3.2).  Returns
    (W, flags)."""
    L = _f64(L)
    B = _f64(B)
    vec = B.ndim == 1
    if vec:
        B = B[:, None].copy()
    d, c = B.shape
    W = np.zeros((d, c))
    fl = _load().orc_solve(d, c, _p(L), _p(B), _p(W))
    return (W[:, 0] if vec else W), int(fl)


def holdout_sse(Xv, Yv, W) -> float:
    """sum((Y_v - X_v W)^2)."""
    Xv = _f64(Xv)
    Yv = _f64(Yv)
    W = _f64(W)
    if Yv.ndim == 1:
        Yv = Yv[:, None].copy()
    if W.ndim == 1:
        W = W[:, None].copy()
    nv, d = Xv.shape
    c = Yv.shape[1]
    return float(_load().orc_holdout_sse(nv, d, c, _p(Xv), d, _p(Yv), c,
                                         _p(W)))


def holdout_sst(Yv) -> float:
    Yv = _f64(Yv)
    if Yv.ndim == 1:
        Yv = Yv[:, None].copy()
    nv, c = Yv.shape
    return float(_load().orc_holdout_sst(nv, c, _p(Yv), c))


def factor_nrmse(Lhat, L) -> float:
    """NRMSE of a fitted factor against the exact one (the paper's NRMSE
    section): sqrt(sum (Lhat - L)^2) / sqrt(sum (L - mean L)^2) over the
    entries i >= j of dense d x d lower factors."""
    Lhat = _f64(Lhat)
    L = _f64(L)
    d = L.shape[0]
    if Lhat.shape != (d, d) or L.shape != (d, d):
        raise ValueError("factor_nrmse takes two d x d matrices")
    return float(_load().orc_factor_nrmse(d, _p(Lhat), _p(L)))


def cv_nrmse(Y, k: int, sse) -> np.ndarray:
    """Hold-out NRMSE per (fold, lambda) from the summed squared residuals
    sse (k x q): sqrt(sse / SST_f), SST_f the squared deviations of fold f's
    labels from their column means.  Predicting every label by its fold's
    column mean gives 1."""
    Y = _f64(Y)
    if Y.ndim == 1:
        Y = Y[:, None].copy()
    b = fold_bounds(Y.shape[0], k)
    sst = np.array([holdout_sst(Y[b[f]:b[f + 1]]) for f in range(k)])
    return np.sqrt(np.asarray(sse, dtype=np.float64) / sst[:, None])


# ---------------------------------------------------------------- pipelines

def refine(H, lam: float, L, B, W, steps: int):
    """Iterative refinement of (H + lam I) W = B with the factor L: returns
    the refined copy of W and the OR of the correction solves' flags."""
    H = _f64(H)
    L = _f64(L)
    B = _f64(B)
    Wr = np.array(W, dtype=np.float64, copy=True, order="C")
    if B.ndim == 1:
        B = B[:, None].copy()
        Wr = Wr.reshape(-1, 1)
    d, c = B.shape
    fl = _load().orc_refine(d, c, _p(H), float(lam), _p(L), _p(B), _p(Wr),
                            int(steps))
    return Wr.reshape(np.shape(W)), int(fl)


def evaluate_deriv(Theta, lam: float, lam_ref: float, basis: int = 0) -> np.ndarray:
    """d Lhat / d lambda of the fitted polynomials (packed vector)."""
    Theta = _f64(Theta)
    r = Theta.shape[0] - 1
    D = Theta.shape[1]
    out = np.zeros(D)
    _load().orc_eval_deriv(D, r, _p(Theta), float(lam), float(lam_ref), _p(out),
                           int(basis))
    return out


def cv_grad(X, Y, k: int, lam_grid, lam_s=None, r: int = 0,
            lam_ref: float | None = None, normalize: bool = True,
            basis: int = 0) -> dict:
    """Hold-out error and its derivative with respect to log lambda at every
    grid value and fold: piCholesky when lam_s is given (degree r), the
    exact method otherwise."""
    X = _f64(X)
    Y = _f64(Y)
    if Y.ndim == 1:
        Y = Y[:, None].copy()
    lam_grid = _f64(lam_grid)
    interp = lam_s is not None
    lam_s = _f64(lam_s) if interp else np.zeros(1)
    if lam_ref is None:
        lam_ref = float(np.max(lam_s)) if interp else 1.0
    n, d = X.shape
    c = Y.shape[1]
    g = lam_s.shape[0]
    q = lam_grid.shape[0]
    mse = np.zeros((k, q))
    dlog = np.zeros((k, q))
    info = np.zeros((k, g if interp else q), dtype=np.int32)
    flags = np.zeros((k, q), dtype=np.int32)
    rc = _load().orc_cv_grad(n, d, c, k, g, r, q, int(normalize), int(interp),
                             _p(X), _p(Y), _p(lam_s), _p(lam_grid), float(lam_ref),
                             _p(mse), _p(dlog), _p(info), _p(flags), int(basis))
    if rc != 0:
        raise ValueError("oracle cv_grad rejected its arguments")
    return {"mse": mse, "dlog": dlog, "info": info, "flags": flags}


def cv_exact(X, Y, k: int, lam_grid, normalize: bool = True,
             want_W: bool = False, refine: int = 0) -> dict:
    """k-fold CV with an exact Cholesky factorization at every grid value
    (then `refine` steps of iterative refinement per solve)."""
    X = _f64(X)
    Y = _f64(Y)
    if Y.ndim == 1:
        Y = Y[:, None].copy()
    lam_grid = _f64(lam_grid)
    n, d = X.shape
    c = Y.shape[1]
    q = lam_grid.shape[0]
    mse = np.zeros((k, q))
    sse = np.zeros((k, q))
    W = np.zeros((k, q, d, c)) if want_W else None
    info = np.zeros((k, q), dtype=np.int32)
    flags = np.zeros((k, q), dtype=np.int32)
    rc = _load().orc_cv_exact(n, d, c, k, q, int(normalize), _p(X), _p(Y),
                              _p(lam_grid), _p(mse), _p(sse), _p(W),
                              _p(info), _p(flags), int(refine))
    if rc != 0:
        raise ValueError("oracle cv_exact rejected its arguments")
    return {"mse": mse, "sse": sse, "W": W, "info": info, "flags": flags}


def cv_interp(X, Y, k: int, lam_s, lam_grid, r: int, lam_ref: float | None = None,
              normalize: bool = True, want_W: bool = False,
              want_theta: bool = False, refine: int = 0, basis: int = 0) -> dict:
    """k-fold CV with piCholesky: Algorithm 1 on each fold, evaluation at
    every grid value, then the same solves and hold-out errors.  With
    refine > 0, that many steps of iterative refinement against
    H_f + lambda_t I follow each solve (the interpolated factor serves as
    the preconditioner)."""
    X = _f64(X)
    Y = _f64(Y)
    if Y.ndim == 1:
        Y = Y[:, None].copy()
    lam_s = _f64(lam_s)
    lam_grid = _f64(lam_grid)
    if lam_ref is None:
        lam_ref = float(np.max(lam_s))
    n, d = X.shape
    c = Y.shape[1]
    g = lam_s.shape[0]
    q = lam_grid.shape[0]
    D = d * (d + 1) // 2
    mse = np.zeros((k, q))
    sse = np.zeros((k, q))
    W = np.zeros((k, q, d, c)) if want_W else None
    Theta = np.zeros((k, r + 1, D)) if want_theta else None
    info = np.zeros((k, g), dtype=np.int32)
    flags = np.zeros((k, q), dtype=np.int32)
    rc = _load().orc_cv_interp(n, d, c, k, g, r, q, int(normalize), _p(X),
                               _p(Y), _p(lam_s), _p(lam_grid), float(lam_ref),
                               _p(mse), _p(sse), _p(W), _p(Theta), _p(info),
                               _p(flags), int(refine), int(basis))
    if rc != 0:
        raise ValueError("oracle cv_interp rejected its arguments")
    return {"mse": mse, "sse": sse, "W": W, "theta": Theta, "info": info,
            "flags": flags}


def fold_interp(H, B, Xv, Yv, lam_s, lam_grid, r: int,
                lam_ref: float | None = None, want_W: bool = False,
                refine: int = 0, basis: int = 0) -> dict:
    """The per-fold piCholesky path starting from that fold's H_f (both
    triangles) and B_f."""
    H = _f64(H)
    B = _f64(B)
    Xv = _f64(Xv)
    Yv = _f64(Yv)
    if B.ndim == 1:
        B = B[:, None].copy()
    if Yv.ndim == 1:
        Yv = Yv[:, None].copy()
    lam_s = _f64(lam_s)
    lam_grid = _f64(lam_grid)
    if lam_ref is None:
        lam_ref = float(np.max(lam_s))
    d = H.shape[0]
    c = B.shape[1]
    g = lam_s.shape[0]
    q = lam_grid.shape[0]
    nv = Xv.shape[0]
    mse = np.zeros(q)
    W = np.zeros((q, d, c)) if want_W else None
    info = np.zeros(g, dtype=np.int32)
    flags = np.zeros(q, dtype=np.int32)
    rc = _load().orc_fold_interp(d, c, g, r, q, _p(H), _p(B), nv, _p(Xv), d,
                                 _p(Yv), c, _p(lam_s), _p(lam_grid),
                                 float(lam_ref), _p(mse), _p(W), _p(info),
                                 _p(flags), int(refine), int(basis))
    if rc != 0:
        raise ValueError("oracle fold_interp rejected its arguments")
    return {"mse": mse, "W": W, "info": info, "flags": flags}


def fold_exact(H, B, Xv, Yv, lam_grid, want_W: bool = False) -> dict:
    """The exact method on one fold from its H_f (both triangles) and B_f:
    at each grid value the Cholesky factor of H_f + lambda I, the forward and
    back substitutions (Sec. 3.2) and the hold-out error of the validation
    rows, composed from cholesky, solve and holdout_sse above.  The grid
    values run on a thread pool (the C calls release the interpreter lock).
    A failed factorization gives info = j+1, NaN results and flags bit0."""
    import concurrent.futures
    H = _f64(H)
    B = _f64(B)
    Xv = _f64(Xv)
    Yv = _f64(Yv)
    if B.ndim == 1:
        B = B[:, None].copy()
    if Yv.ndim == 1:
        Yv = Yv[:, None].copy()
    lam_grid = _f64(lam_grid)
    d, c = B.shape
    q = lam_grid.shape[0]
    nv = Xv.shape[0]
    mse = np.zeros(q)
    W = np.zeros((q, d, c)) if want_W else None
    info = np.zeros(q, dtype=np.int32)
    flags = np.zeros(q, dtype=np.int32)

    def unit(t):
        L, inf = cholesky(H, float(lam_grid[t]))
        info[t] = inf
        if inf != 0:
            mse[t] = np.nan
            flags[t] = 1
            if want_W:
                W[t] = np.nan
            return
        Wt, fl = solve(L, B)
        sse = holdout_sse(Xv, Yv, Wt)
        if not np.isfinite(sse):
            fl |= 1
        flags[t] = fl
        mse[t] = sse / (nv * c)
        if want_W:
            W[t] = Wt

    with concurrent.futures.ThreadPoolExecutor(max(1, min(q, num_threads()))) as ex:
        list(ex.map(unit, range(q)))
    return {"mse": mse, "W": W, "info": info, "flags": flags}


# ---------------------------------------------------------------- vectorisation orders (Sec. 5)

def recursive_order(h: int, h0: int) -> list:
    """The (row, column) entries of an order-h lower triangle in the order
    of the recursive vectorisation (Sec. 5, eq. recursive): the square
    block L12 (rows h/2..h-1, columns 0..h/2-1) row by row, then the
    triangle L11, then the triangle L22, each split the same way until its
    order is at most h0, where the rows are concatenated."""
    def rec(r0, h):
        if h <= h0:
            return [(r0 + i, r0 + j) for i in range(h) for j in range(i + 1)]
        half = h // 2
        l12 = [(r0 + half + i, r0 + j) for i in range(h - half) for j in range(half)]
        return l12 + rec(r0, half) + rec(r0 + half, h - half)
    return rec(0, h)


# ---------------------------------------------------------------- the paper's variants (Sec. 6.2, 6.5)

def pinrmse(X, Y, k: int, lam_s, lam_grid, r: int, lam_ref: float | None = None,
            normalize: bool = True) -> dict:
    """PINRMSE (Sec. 6.5): Algorithm 1 with the g x D matrix T replaced by
    the g-vector of exact hold-out errors at the samples, fold by fold; the
    fitted polynomial is evaluated at the grid."""
    lam_s = _f64(lam_s)
    lam_grid = _f64(lam_grid)
    if lam_ref is None:
        lam_ref = float(np.max(lam_s))
    ex = cv_exact(X, Y, k, lam_s, normalize=normalize)
    mse = np.zeros((k, lam_grid.shape[0]))
    for f in range(k):
        t = ex["mse"][f][:, None].copy()          # g x 1 in place of T
        theta = fit(t, lam_s, r, lam_ref)          # (r+1) x 1
        for j, lam in enumerate(lam_grid):
            mse[f, j] = evaluate(theta, lam, lam_ref)[0]
    return {"mse": mse, "mse_samples": ex["mse"], "info": ex["info"],
            "flags": ex["flags"]}


def mchol(X, Y, k: int, c0: float, s: float = 1.5, s0: float = 0.0025,
          normalize: bool = True) -> dict:
    """Multi-level Cholesky search (MChol, Sec. 6.2): starting from the
    range [10^(c-s), 10^(c+s)], evaluate the fold-mean hold-out error with
    exact factors at 10^(c-s), 10^c, 10^(c+s), move c to the best of the
    three (ties: the smallest lambda), halve s, and stop once s <= s0.
    Returns the final lambda = 10^c and the visited points."""
    c = float(c0)
    trace = []
    while True:
        lams = 10.0 ** np.array([c - s, c, c + s])
        cvv = cv_exact(X, Y, k, lams, normalize=normalize)["mse"].mean(axis=0)
        j = int(np.argmin(cvv))
        trace.append((lams, cvv))
        c = float(np.log10(lams[j]))
        s = s / 2.0
        if s <= s0:
            break
    return {"lam": 10.0 ** c, "log10_lam": c, "trace": trace}


# ---------------------------------------------------------------- selection (Sec. 6)

def cv_curve(mse) -> np.ndarray:
    """Unweighted mean hold-out error over folds, per grid value."""
    return np.asarray(mse, dtype=np.float64).mean(axis=0)


def select(curve) -> int:
    """Index of the minimum of the CV curve; ties go to the smallest index
    (smallest lambda).  Non-finite entries never win."""
    c = np.asarray(curve, dtype=np.float64)
    c = np.where(np.isfinite(c), c, np.inf)
    return int(np.argmin(c))


def gaps(curve_pi, curve_ex, lam_grid) -> dict:
    """Accuracy of the interpolated curve against the exact one (Sec. 6.4):
    largest relative curve gap, relative gap of the minima, regret of the
    selected value, and |log10| ratio of the selected lambdas."""
    cp = np.asarray(curve_pi, dtype=np.float64)
    ce = np.asarray(curve_ex, dtype=np.float64)
    lam = np.asarray(lam_grid, dtype=np.float64)
    tp, te = select(cp), select(ce)
    return {
        "curve_gap": float(np.max(np.abs(cp - ce) / np.abs(ce))),
        "min_gap": float((cp.min() - ce.min()) / ce.min()),
        "regret": float(ce[tp] - ce.min()),
        "sel_err_log10": float(abs(np.log10(lam[tp] / lam[te]))),
        "t_pi": tp,
        "t_ex": te,
    }
