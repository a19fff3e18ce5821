"""Helpers for the GPU tests: run library entry points through the C-ABI
binding with torch-allocated device buffers, and convert the tile-packed
layout to dense arrays on the host for comparison with the oracle."""
from __future__ import annotations

import numpy as np
import torch

from paper_1404_0466_amd import binding as B

NB = B.NB
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def empty(n, dtype=torch.float64):
    return torch.empty(int(n), dtype=dtype, device=DEV)


def ws(nbytes):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=DEV)


def unpack(P, d, nmat):
    """Packed device triangles -> (nmat, d, d) host lower triangles."""
    A = empty(nmat * d * d)
    B.pichol_unpack(d, nmat, P, A, d)
    torch.cuda.synchronize()
    return A.cpu().numpy().reshape(nmat, d, d)


def pack(A, d):
    """(nmat, d, d) host symmetric/lower matrices -> packed device."""
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(-1, d, d)
    nmat = A.shape[0]
    P = empty(nmat * B.pichol_packed_elems(d))
    B.pichol_pack(d, nmat, dev(A.reshape(-1)), d, P)
    return P


def slab_to_w(Z, d, nmat, q, c):
    W = empty(nmat * q * d * c)
    B.pichol_slab_to_weights(d, nmat, q, c, Z, W)
    torch.cuda.synchronize()
    return W.cpu().numpy().reshape(nmat, q, d, c)


def fold_sizes(n, k):
    return np.array([len(a) for a in np.array_split(np.arange(n), k)], dtype=np.int64)


def gram(X, Y, k, normalize=True):
    n, d = X.shape
    c = Y.shape[1]
    p = B.make_problem(n, d, c, k, normalize=normalize)
    dp = B.pichol_padded_order(d)
    S = B.pichol_packed_elems(d)
    out = {
        "G": empty(k * dp * dp), "C": empty(k * dp * c), "yy": empty(k),
        "H": empty(k * S), "B": empty(k * dp * c),
    }
    B.pichol_gram(p, dev(X), dev(Y), out["G"], out["C"], out["yy"], out["H"],
                  out["B"])
    return out


def cv(prob, method, X=None, Y=None, lam_s=None, lam_grid=None, r=None,
       want_W=True, normalize=True, k=None, precision=0, refine=0, basis=0):
    """Run the pipeline (gram + interp or exact) on the GPU."""
    X = prob.X if X is None else X
    Y = prob.Y if Y is None else Y
    lam_s = prob.lam_s if lam_s is None else np.asarray(lam_s)
    lam_grid = prob.lam_grid if lam_grid is None else np.asarray(lam_grid)
    r = prob.r if r is None else r
    k = prob.k if k is None else k
    n, d = X.shape
    c = Y.shape[1]
    g, q = len(lam_s), len(lam_grid)
    p = B.make_problem(n, d, c, k, g, r, q, normalize, precision=precision,
                       refine=refine, basis=basis)
    m = B.PICHOL_METHOD_INTERP if method == "interp" else B.PICHOL_METHOD_EXACT
    nbytes = B.pichol_workspace_size(p, m)
    w = ws(nbytes)
    err = empty(k * q)
    W = empty(k * q * d * c) if want_W else None
    flags = empty(k * q, torch.int32)
    Xd, Yd = dev(X), dev(Y)
    if method == "interp":
        info = empty(k * g, torch.int32)
        B.pichol_cv(p, Xd, Yd, lam_s, lam_grid, float(np.max(lam_s)), w, nbytes,
                    err, W, info, flags)
    else:
        info = empty(k * q, torch.int32)
        B.pichol_exact_cv(p, Xd, Yd, lam_grid, w, nbytes, err, W, info, flags)
    torch.cuda.synchronize()
    return {
        "mse": err.cpu().numpy().reshape(k, q),
        "W": W.cpu().numpy().reshape(k, q, d, c) if want_W else None,
        "info": info.cpu().numpy().reshape(k, -1),
        "flags": flags.cpu().numpy().reshape(k, q),
    }


class BatchRun:
    """Device buffers and the ctypes batch for a list of workloads.Problem
    (pichol_cv_batch)."""

    def __init__(self, probs, method, precision=0, want_W=True, basis=0):
        self.probs = probs
        self.method = B.PICHOL_METHOD_INTERP if method == "interp" else B.PICHOL_METHOD_EXACT
        self.interp = method == "interp"
        self.want_W = want_W
        self.bufs = []
        ents = []
        for p in probs:
            k, q = p.k, p.q
            nf = p.g if self.interp else q
            b = {
                "X": dev(p.X), "Y": dev(p.Y), "err": empty(k * q),
                "W": empty(k * q * p.d * p.c) if want_W else None,
                "info": empty(k * nf, torch.int32), "flags": empty(k * q, torch.int32),
            }
            self.bufs.append(b)
            ents.append(dict(p=B.make_problem(p.n, p.d, p.c, k, p.g, p.r, q, True,
                                              precision=precision, basis=basis),
                             lam_s=p.lam_s if self.interp else None,
                             lam_grid=p.lam_grid, lam_ref=p.lam_ref, **b))
        self.batch = B.Batch(ents)
        self.nbytes = B.pichol_batch_workspace_size(self.batch, self.method)
        self.ws = ws(self.nbytes)

    def run(self, tune=None):
        B.pichol_cv_batch(self.batch, self.method, tune, self.ws, self.nbytes)
        torch.cuda.synchronize()
        return self.results()

    def clear(self):
        for b in self.bufs:
            b["err"].fill_(float("nan"))
            b["info"].fill_(-7)
            b["flags"].fill_(-7)
            if b["W"] is not None:
                b["W"].fill_(float("nan"))
        torch.cuda.synchronize()

    def results(self):
        out = []
        for p, b in zip(self.probs, self.bufs):
            out.append({
                "mse": b["err"].cpu().numpy().reshape(p.k, p.q),
                "W": b["W"].cpu().numpy().reshape(p.k, p.q, p.d, p.c) if self.want_W else None,
                "info": b["info"].cpu().numpy().reshape(p.k, -1),
                "flags": b["flags"].cpu().numpy().reshape(p.k, p.q),
            })
        return out


def library_fit_solve(H, lam_s, lam_ref, r, lam, Bd):
    """The interpolated solve composed from library routines: LAPACK
    Cholesky at the samples, a least-squares fit of every entry in
    tau = lambda/lam_ref by LAPACK (SVD based, accurate to cond(V) eps, not
    cond(V)^2 eps as the normal equations), evaluation, and LAPACK
    triangular solves."""
    import scipy.linalg
    d = H.shape[0]
    g = len(lam_s)
    Ls = np.stack([np.linalg.cholesky(H + l * np.eye(d)) for l in lam_s])
    V = np.vander(np.asarray(lam_s) / lam_ref, r + 1, increasing=True)
    coef, *_ = np.linalg.lstsq(V, Ls.reshape(g, -1), rcond=None)
    out = []
    for l in lam:
        L = np.tril((np.vander([l / lam_ref], r + 1, increasing=True)[0] @ coef)
                    .reshape(d, d))
        z = scipy.linalg.solve_triangular(L, Bd, lower=True)
        out.append(scipy.linalg.solve_triangular(L.T, z, lower=False))
    return np.stack(out)
