"""The paper's other search procedures, as drivers over the library's
pipeline calls (no kernels of their own beyond those calls).

mchol    Multi-level Cholesky (MChol, Sec. 6.2): a bracketing search over
         log10 lambda with exact factorizations at three points per level.
pinrmse  PINRMSE (Sec. 6.5): the hold-out errors at the g samples
         interpolated directly (pichol_cv_pinrmse).
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def mchol(X, Y, k: int, c0: float, s: float = 1.5, s0: float = 0.0025,
          normalize: bool = True, precision: int = B.PICHOL_PREC_FP64) -> dict:
    """X, Y: device float64 tensors (n x d, n x c).  Starting from the range
    [10^(c0-s), 10^(c0+s)]: evaluate the fold-mean hold-out error with exact
    Cholesky factors at 10^(c-s), 10^c and 10^(c+s) (one pichol_cv_exact
    call of three grid values), recentre c on the best point (ties: the
    smallest lambda), halve s, stop once s <= s0.  Returns the final lambda,
    the visited points and their errors, and the number of exact
    factorizations made."""
    n, d = X.shape
    c = Y.shape[1]
    p = B.make_problem(n, d, c, k, 1, 0, 3, normalize, precision=precision)
    nbytes = B.pichol_workspace_size(p, B.PICHOL_METHOD_EXACT)
    dev = X.device
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    err = torch.empty(k * 3, dtype=torch.float64, device=dev)
    info = torch.empty(k * 3, dtype=torch.int32, device=dev)
    flags = torch.empty(k * 3, dtype=torch.int32, device=dev)
    B.pichol_cv_gram(p, X.contiguous(), Y.contiguous(), ws, nbytes)
    cc = float(c0)
    trace = []
    nfac = 0
    while True:
        lams = 10.0 ** np.array([cc - s, cc, cc + s])
        B.pichol_cv_exact(p, lams, ws, nbytes, err, None, info, flags)
        nfac += 3 * k
        cvv = err.view(k, 3).mean(0).cpu().numpy()
        if int(info.max()) != 0:
            raise RuntimeError("a shifted matrix was not positive definite")
        j = int(np.argmin(cvv))
        trace.append((lams, cvv))
        cc = float(np.log10(lams[j]))
        s = s / 2.0
        if s <= s0:
            break
    return {"lam": 10.0 ** cc, "log10_lam": cc, "trace": trace,
            "factorizations": nfac}


def pinrmse(X, Y, k: int, lam_s, lam_grid, r: int, lam_ref: float | None = None,
            normalize: bool = True) -> dict:
    """Hold-out errors at lam_grid from a degree-r fit to the exact errors
    at the samples lam_s (pichol_cv_pinrmse).  Returns the k x q curve and
    the k x g sample errors."""
    n, d = X.shape
    c = Y.shape[1]
    lam_s = np.asarray(lam_s, dtype=np.float64)
    lam_grid = np.asarray(lam_grid, dtype=np.float64)
    g, q = lam_s.shape[0], lam_grid.shape[0]
    lam_ref = float(np.max(lam_s)) if lam_ref is None else float(lam_ref)
    p = B.make_problem(n, d, c, k, g, r, q, normalize)
    nbytes = B.pichol_workspace_size(p, B.PICHOL_METHOD_PINRMSE)
    dev = X.device
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    err = torch.empty(k * q, dtype=torch.float64, device=dev)
    err_s = torch.empty(k * g, dtype=torch.float64, device=dev)
    info = torch.empty(k * g, dtype=torch.int32, device=dev)
    flags = torch.empty(k * g, dtype=torch.int32, device=dev)
    B.pichol_cv_gram(p, X.contiguous(), Y.contiguous(), ws, nbytes)
    B.pichol_cv_pinrmse(p, lam_s, lam_grid, lam_ref, ws, nbytes, err, err_s, info,
                        flags)
    return {"mse": err.view(k, q).cpu().numpy(), "mse_samples": err_s.view(k, g).cpu().numpy(),
            "info": info.view(k, g).cpu().numpy(), "flags": flags.view(k, g).cpu().numpy()}
