"""Edge cases of the pipeline calls against the oracle: unnormalised Gram
matrices (the paper's X^T X), strided X rows (ldx > d), two folds and many
folds, a single right-hand side and a single grid value, more than 16
right-hand sides, order-1 problems,
interpolation through every sample (r = g - 1) and the smallest batch."""
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


def _check(got, want, rtol=1e-10):
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=rtol, atol=0)


@pytest.mark.parametrize("method", ["interp", "exact"])
def test_unnormalised_gram(gu, method):
    p = workloads.gaussian_problem(500, 140, 2, seed=41, g=4, q=6)
    scale = p.n * 0.8  # shifts of the order of X^T X's entries
    lam_s, lam_g = p.lam_s * scale, p.lam_grid * scale
    got = gu.cv(p, method, lam_s=lam_s, lam_grid=lam_g, normalize=False)
    if method == "interp":
        want = oracle.cv_interp(p.X, p.Y, p.k, lam_s, lam_g, p.r, normalize=False)
    else:
        want = oracle.cv_exact(p.X, p.Y, p.k, lam_g, normalize=False)
    _check(got, want)


@pytest.mark.parametrize("k", [2, 7])
def test_fold_counts(gu, k):
    p = workloads.gaussian_problem(503, 130, 3, seed=42 + k, g=4, q=5, k=k)
    got = gu.cv(p, "interp")
    want = oracle.cv_interp(p.X, p.Y, k, p.lam_s, p.lam_grid, p.r, want_W=True)
    _check(got, want)


def test_single_rhs_single_lambda(gu):
    p = workloads.gaussian_problem(300, 129, 1, seed=44, g=3, r=2, q=1)
    for method in ["interp", "exact"]:
        got = gu.cv(p, method)
        want = (oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r) if method == "interp"
                else oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid))
        _check(got, want)


@pytest.mark.parametrize("c", [17, 40])
def test_many_right_hand_sides(gu, c):
    """More than 16 label columns: the Gram right-hand sides, the diagonal
    applies and the exact-factor updates loop over 16-column groups; the
    interpolated update covers several 128-column slab blocks per lambda."""
    p = workloads.gaussian_problem(700, 200, c, seed=50 + c, g=4, q=7)
    for method in ["interp", "exact"]:
        got = gu.cv(p, method)
        want = (oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True)
                if method == "interp" else
                oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid, want_W=True))
        _check(got, want)
        np.testing.assert_allclose(got["W"], want["W"], rtol=1e-8, atol=1e-12)


def test_order_one_problem(gu):
    p = workloads.gaussian_problem(60, 1, 2, seed=45, g=2, r=1, q=3)
    got = gu.cv(p, "interp")
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, 1, want_W=True)
    _check(got, want)
    np.testing.assert_allclose(got["W"], want["W"], rtol=1e-10, atol=0)


def test_strided_rows(gu):
    """X and Y given with leading dimensions larger than d and c."""
    B = gu.B
    p = workloads.gaussian_problem(400, 150, 3, seed=46, g=4, q=5)
    n, d, c, k, g, q = p.n, p.d, p.c, p.k, p.g, p.q
    Xw = np.zeros((n, d + 5))
    Xw[:, :d] = p.X
    Xw[:, d:] = 7.0  # must not be read
    Yw = np.zeros((n, c + 2))
    Yw[:, :c] = p.Y
    Yw[:, c:] = -3.0
    prob = B.make_problem(n, d, c, k, g, p.r, q, True, ldx=d + 5, ldy=c + 2)
    nb = B.pichol_workspace_size(prob, B.PICHOL_METHOD_INTERP)
    err, info = gu.empty(k * q), gu.empty(k * g, torch.int32)
    flags = gu.empty(k * q, torch.int32)
    B.pichol_cv(prob, gu.dev(Xw), gu.dev(Yw), p.lam_s, p.lam_grid, p.lam_ref, gu.ws(nb), nb,
                err, None, info, flags)
    torch.cuda.synchronize()
    want = oracle.cv_interp(p.X, p.Y, k, p.lam_s, p.lam_grid, p.r)
    got = {"mse": err.cpu().numpy().reshape(k, q), "info": info.cpu().numpy(),
           "flags": flags.cpu().numpy()}
    _check(got, want)


def test_interpolation_through_every_sample(gu):
    """r = g - 1: the fitted factor passes through every exact sample
    factor, so at grid values equal to samples piCholesky gives the exact
    errors."""
    p = workloads.gaussian_problem(500, 200, 3, seed=47, g=4, r=3, q=10,
                                   lam_range=(1e-3, 1.0))
    lam_s = p.lam_grid[[0, 3, 6, 9]]
    gi = gu.cv(p, "interp", lam_s=lam_s, r=3)
    ge = gu.cv(p, "exact")
    tau = lam_s / lam_s.max()
    cond = np.linalg.cond(np.vander(tau, 4, increasing=True))
    np.testing.assert_allclose(gi["mse"][:, [0, 3, 6, 9]], ge["mse"][:, [0, 3, 6, 9]],
                               rtol=max(1e-10, 100 * cond * np.finfo(float).eps))


def test_batch_of_one(gu):
    p = workloads.gaussian_problem(300, 100, 2, seed=48, g=4, q=5)
    run = gu.BatchRun([p], "interp")
    got = run.run()[0]
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
    _check(got, want)


@pytest.mark.parametrize("r", [2, 3])
def test_log_lambda_basis(gu, r):
    """Polynomials in log(lambda / lam_ref) instead of lambda / lam_ref:
    the pipeline, the batch call and PINRMSE follow the oracle's log-basis
    fit."""
    p = workloads.gaussian_problem(1003, 300, 3, seed=50 + r, g=5, r=r, q=11)
    got = gu.cv(p, "interp", basis=1)
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, r, want_W=True, basis=1)
    u = np.log(p.lam_s / p.lam_ref)
    cond = np.linalg.cond(np.vander(u, r + 1, increasing=True))
    tol = max(1e-10, 10 * cond ** 2 * np.finfo(float).eps)
    _check(got, want, rtol=tol)
    run = gu.BatchRun([p], "interp", basis=1)
    np.testing.assert_array_equal(run.run()[0]["mse"], got["mse"])
    # the two bases differ (the interpolation is not the same function)
    lin = gu.cv(p, "interp", want_W=False)
    assert np.max(np.abs(lin["mse"] - got["mse"]) / got["mse"]) > 1e-8


def test_log_basis_rejects_nonpositive_lambda(gu):
    B = gu.B
    p = workloads.gaussian_problem(300, 100, 2, seed=52, g=4, q=5)
    prob = B.make_problem(p.n, p.d, p.c, p.k, p.g, p.r, p.q, True, basis=1)
    nb = B.pichol_workspace_size(prob, B.PICHOL_METHOD_INTERP)
    w = gu.ws(nb)
    B.pichol_cv_gram(prob, gu.dev(p.X), gu.dev(p.Y), w, nb)
    lam_grid = p.lam_grid.copy()
    lam_grid[0] = 0.0
    with pytest.raises(B.PicholError) as e:
        B.pichol_cv_interp(prob, p.lam_s, lam_grid, p.lam_ref, w, nb, gu.empty(p.k * p.q),
                           None, gu.empty(p.k * p.g, torch.int32),
                           gu.empty(p.k * p.q, torch.int32))
    assert e.value.status == B.PICHOL_ERR_ARG



@pytest.mark.parametrize("k,g", [(64, 4), (5, 32)])
def test_largest_fold_and_sample_counts(gu, k, g):
    """The boundary's limits on the problem: 64 folds (the hold-out
    normalisation and the fold split hold 64 entries), 32 samples (the
    fit's pseudo-inverse holds 32 columns)."""
    p = workloads.gaussian_problem(640, 96, 2, seed=60 + k + g, g=g, r=2, q=6, k=k)
    got = gu.cv(p, "interp")
    want = oracle.cv_interp(p.X, p.Y, k, p.lam_s, p.lam_grid, p.r, want_W=True)
    _check(got, want)
    ge = gu.cv(p, "exact")
    we = oracle.cv_exact(p.X, p.Y, k, p.lam_grid, want_W=True)
    _check(ge, we)


def test_largest_degree(gu):
    """Degree 7 (eight planes, the largest the fit takes) from eight samples
    over one decade, against the same steps composed from LAPACK routines
    (cond(V) = 7e5 in tau: the oracle's normal equations would lose
    cond(V)^2 eps; two backward-stable fits evaluated inside the sampled
    range meet far closer)."""
    import gpu_util
    p = workloads.gaussian_problem(900, 120, 3, seed=71, k=3, g=8, q=9,
                                   lam_range=(1e-1, 1.0))
    lam_s = np.logspace(np.log10(p.lam_grid[0]), np.log10(p.lam_grid[-1]), 8)
    got = gu.cv(p, "interp", lam_s=lam_s, r=7)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    b = oracle.fold_bounds(p.n, p.k)
    for f in range(p.k):
        mask = np.ones(p.n, bool)
        mask[b[f]:b[f + 1]] = False
        Xt, Yt, Xv, Yv = p.X[mask], p.Y[mask], p.X[~mask], p.Y[~mask]
        ntr = mask.sum()
        W = gpu_util.library_fit_solve(Xt.T @ Xt / ntr, lam_s, lam_s.max(), 7,
                                       p.lam_grid, Xt.T @ Yt / ntr)
        for t in range(len(p.lam_grid)):
            mse = np.sum((Yv - Xv @ W[t]) ** 2) / Yv.size
            assert abs(got["mse"][f, t] - mse) <= 1e-9 * mse, (f, t)
