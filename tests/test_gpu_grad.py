"""Differentiation form: d(hold-out error)/d(log lambda) through the
interpolated factor (pichol_cv_interp_grad) and through exact factors
(pichol_cv_exact_grad), against the oracle's adjoint formula (itself pinned
by central differences and the SVD form), against central differences of
the GPU's own forward pass, and through the torch.autograd wrapper.

Tolerance: the derivative is compared relative to the largest |dlog| of the
curve (it changes sign at the minimum); 1e-9 against the FP64 oracle,
1e-6 against central differences with h = 1e-4 in log lambda (truncation
O(h^2) ~ 1e-8 relative, rounding eps * mse / h ~ 1e-12).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


def gpu_grad(gu, prob, method, lam_grid=None, basis=0):
    B = gu.B
    lam_grid = prob.lam_grid if lam_grid is None else np.asarray(lam_grid)
    n, d, c, k, g, q = prob.n, prob.d, prob.c, prob.k, prob.g, len(lam_grid)
    p = B.make_problem(n, d, c, k, g, prob.r, q, True, basis=basis)
    m = (B.PICHOL_METHOD_INTERP if method == "interp" else B.PICHOL_METHOD_EXACT)
    nb = B.pichol_workspace_size(p, m | B.PICHOL_METHOD_GRAD)
    w = gu.ws(nb)
    err, dlog = gu.empty(k * q), gu.empty(k * q)
    flags = gu.empty(k * q, torch.int32)
    B.pichol_cv_gram(p, gu.dev(prob.X), gu.dev(prob.Y), w, nb)
    if method == "interp":
        info = gu.empty(k * g, torch.int32)
        B.pichol_cv_interp_grad(p, prob.lam_s, lam_grid, prob.lam_ref, w, nb, err,
                                dlog, None, info, flags)
    else:
        info = gu.empty(k * q, torch.int32)
        B.pichol_cv_exact_grad(p, lam_grid, w, nb, err, dlog, None, info, flags)
    torch.cuda.synchronize()
    return {"mse": err.cpu().numpy().reshape(k, q), "dlog": dlog.cpu().numpy().reshape(k, q),
            "info": info.cpu().numpy(), "flags": flags.cpu().numpy().reshape(k, q)}


PROBS = [dict(n=1100, d=300, c=3, seed=4, g=5, q=11),
         dict(n=700, d=129, c=1, seed=8, g=4, q=7)]


@pytest.mark.parametrize("cfg", PROBS)
def test_interp_grad_matches_oracle(gu, cfg):
    cfg = dict(cfg)
    n, d, c = cfg.pop("n"), cfg.pop("d"), cfg.pop("c")
    prob = workloads.gaussian_problem(n, d, c, r=2, **cfg)
    got = gpu_grad(gu, prob, "interp")
    want = oracle.cv_grad(prob.X, prob.Y, prob.k, prob.lam_grid, prob.lam_s, prob.r)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=1e-10, atol=0)
    scale = np.abs(want["dlog"]).max()
    assert np.abs(got["dlog"] - want["dlog"]).max() <= 1e-9 * scale


def test_exact_grad_matches_oracle(gu):
    prob = workloads.gaussian_problem(1100, 300, 3, seed=4, g=5, r=2, q=11)
    got = gpu_grad(gu, prob, "exact")
    want = oracle.cv_grad(prob.X, prob.Y, prob.k, prob.lam_grid)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=1e-10, atol=0)
    scale = np.abs(want["dlog"]).max()
    assert np.abs(got["dlog"] - want["dlog"]).max() <= 1e-9 * scale


def test_interp_grad_matches_gpu_central_differences(gu):
    prob = workloads.gaussian_problem(1100, 300, 3, seed=4, g=5, r=2, q=11)
    got = gpu_grad(gu, prob, "interp")
    h = 1e-4
    up = gu.cv(prob, "interp", lam_grid=prob.lam_grid * np.exp(h), want_W=False)["mse"]
    dn = gu.cv(prob, "interp", lam_grid=prob.lam_grid * np.exp(-h), want_W=False)["mse"]
    fd = (up - dn) / (2 * h)
    assert np.abs(fd - got["dlog"]).max() <= 1e-6 * np.abs(got["dlog"]).max()


def test_autograd_wrapper(gu):
    from paper_1404_0466_amd.autograd import PiCholCV
    prob = workloads.gaussian_problem(700, 129, 2, seed=3, g=4, r=2, q=6)
    X, Y = gu.dev(prob.X), gu.dev(prob.Y)
    f = PiCholCV(X, Y, prob.k, prob.lam_s, prob.r, prob.q)
    log_lam = torch.tensor(np.log(prob.lam_grid), dtype=torch.float64, requires_grad=True)
    err = f(log_lam)
    loss = err.mean(0).sum()
    loss.backward()
    want = oracle.cv_grad(prob.X, prob.Y, prob.k, prob.lam_grid, prob.lam_s, prob.r)
    np.testing.assert_allclose(err.detach().cpu().numpy(), want["mse"], rtol=1e-10)
    g_want = want["dlog"].mean(0)
    assert np.abs(log_lam.grad.numpy() - g_want).max() <= 1e-9 * np.abs(g_want).max()
    # torch's own finite-difference Jacobian check of the wrapper
    ok = torch.autograd.gradcheck(lambda x: f(x), (log_lam.detach().requires_grad_(),),
                                  eps=1e-5, atol=1e-7, rtol=1e-4)
    assert ok


def test_log_basis_grad_matches_oracle(gu):
    prob = workloads.gaussian_problem(900, 260, 3, seed=14, g=5, r=2, q=9)
    got = gpu_grad(gu, prob, "interp", basis=1)
    want = oracle.cv_grad(prob.X, prob.Y, prob.k, prob.lam_grid, prob.lam_s, prob.r, basis=1)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=1e-10, atol=0)
    assert np.abs(got["dlog"] - want["dlog"]).max() <= 1e-9 * np.abs(want["dlog"]).max()

