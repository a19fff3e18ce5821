"""Hold-out error of piCholesky cross-validation as a differentiable function
of log lambda, for continuous lambda search with torch optimisers.

``PiCholCV(X, Y, k, lam_s, r)`` forms the fold Gram matrices once
(pichol_cv_gram).  Calling it with a tensor of q log-lambda values returns
the k x q hold-out errors; their backward pass uses the derivative computed
by pichol_cv_interp_grad in the same forward call (the adjoint of
interpolate -> triangular solves -> hold-out error, in the library's
kernels).  The only arithmetic here is the chain rule's product of the
incoming gradient with that derivative.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class _InterpCV(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_lam, state):
        err, dlog = state.run(log_lam)
        ctx.save_for_backward(dlog)
        ctx.in_device, ctx.in_dtype = log_lam.device, log_lam.dtype
        return err

    @staticmethod
    def backward(ctx, grad_err):
        (dlog,) = ctx.saved_tensors
        g = (grad_err.to(dlog) * dlog).sum(0)
        return g.to(device=ctx.in_device, dtype=ctx.in_dtype), None


class PiCholCV:
    """k-fold piCholesky cross-validation of ridge regression on (X, Y)
    with fixed sample lambdas lam_s and degree r (Algorithm 1), evaluated at
    q lambda values given as log lambda.  X, Y: device float64 tensors
    (n x d, n x c); the grid size q is fixed at construction."""

    def __init__(self, X, Y, k, lam_s, r, q, lam_ref=None, normalize=True,
                 precision=B.PICHOL_PREC_FP64):
        n, d = X.shape
        c = Y.shape[1]
        self.lam_s = np.asarray(lam_s, dtype=np.float64)
        self.lam_ref = float(np.max(self.lam_s)) if lam_ref is None else float(lam_ref)
        self.k, self.q, self.d, self.c = k, q, d, c
        self.p = B.make_problem(n, d, c, k, len(self.lam_s), r, q, normalize,
                                precision=precision)
        self.nbytes = B.pichol_workspace_size(
            self.p, B.PICHOL_METHOD_INTERP | B.PICHOL_METHOD_GRAD)
        dev = X.device
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        self.err = torch.empty(k * q, dtype=torch.float64, device=dev)
        self.dlog = torch.empty(k * q, dtype=torch.float64, device=dev)
        self.info = torch.empty(k * len(self.lam_s), dtype=torch.int32, device=dev)
        self.flags = torch.empty(k * q, dtype=torch.int32, device=dev)
        B.pichol_cv_gram(self.p, X.contiguous(), Y.contiguous(), self.ws, self.nbytes)

    def run(self, log_lam):
        lam = torch.exp(log_lam.detach().to(torch.float64)).cpu().numpy()
        if lam.shape != (self.q,):
            raise ValueError(f"expected {self.q} log-lambda values")
        B.pichol_cv_interp_grad(self.p, self.lam_s, lam, self.lam_ref, self.ws,
                                self.nbytes, self.err, self.dlog, None, self.info,
                                self.flags)
        k, q = self.k, self.q
        return (self.err.view(k, q).clone(), self.dlog.view(k, q).clone())

    def __call__(self, log_lam):
        """k x q hold-out errors, differentiable with respect to log_lam."""
        return _InterpCV.apply(log_lam, self)

    def status(self):
        """(info, flags) of the last call, as host arrays."""
        return self.info.cpu().numpy(), self.flags.cpu().numpy()
