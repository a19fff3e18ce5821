"""Parity at the benchmark's full size: random Fourier features, n=60000,
d=4096, c=10, k=5, g=6, r=2, q=64, in the launch configuration bench.py
times (the pipeline calls through the C-ABI).

The oracle cannot redo the whole job in a test's time, so the checks are
(1) fold 0 of the interpolated cross-validation, which the oracle computes
in full from that fold's Gram matrices (about 20 s on 16 cores), and
(2) the exact baseline at four grid values of fold 0, which the oracle
factors and solves in full, and (3) properties checked entry by entry on
samples: Gram entries against their definition, and L L^T = H + lambda I for
exact factors.  The d = 2048 random-feature workload is compared with the
oracle at every grid value.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big(gpu):
    import gpu_util
    prob = workloads.named("rff_n60000_d4096")
    return gpu_util, prob


def test_fullsize_fold0_matches_oracle(big):
    gu, p = big
    got = gu.cv(p, "interp", want_W=False)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    nv = len(np.array_split(np.arange(p.n), p.k)[0])
    Xt, Yt = p.X[nv:], p.Y[nv:]
    H = Xt.T @ Xt / Xt.shape[0]
    Bm = Xt.T @ Yt / Xt.shape[0]
    want = oracle.fold_interp(H, Bm, p.X[:nv], p.Y[:nv], p.lam_s, p.lam_grid, p.r)
    assert np.all(want["info"] == 0) and np.all(want["flags"] == 0)
    np.testing.assert_allclose(got["mse"][0], want["mse"], rtol=1e-10, atol=0)


def _fold_grams(p, f):
    """H_f, B_f (numpy, from the training rows) and the validation rows."""
    b = oracle.fold_bounds(p.n, p.k)
    mask = np.ones(p.n, bool)
    mask[b[f]:b[f + 1]] = False
    Xt, Yt = p.X[mask], p.Y[mask]
    ntr = mask.sum()
    return Xt.T @ Xt / ntr, Xt.T @ Yt / ntr, p.X[~mask], p.Y[~mask]


def test_fullsize_exact_sampled_against_oracle(big):
    """The exact baseline at full size: the GPU's exact CV (all 320
    factorizations, as bench.py times it) at four grid values of fold 0
    against the oracle's factorization, solves and direct residual there."""
    gu, p = big
    got = gu.cv(p, "exact", want_W=False)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    idx = [0, 21, 42, 63]
    H, Bm, Xv, Yv = _fold_grams(p, 0)
    want = oracle.fold_exact(H, Bm, Xv, Yv, p.lam_grid[idx])
    assert np.all(want["info"] == 0) and np.all(want["flags"] == 0)
    np.testing.assert_allclose(got["mse"][0, idx], want["mse"], rtol=1e-10, atol=0)


def test_fullsize_gram_and_factor_properties(big):
    gu, p = big
    B = gu.B
    n, d, c, k = p.n, p.d, p.c, p.k
    g = gu.gram(p.X, p.Y, k)
    rng = np.random.default_rng(0)
    idx = rng.integers(0, d, size=(40, 2))
    H = gu.unpack(g["H"], d, k)  # lower triangles
    starts = np.concatenate([[0], np.cumsum(gu.fold_sizes(n, k))])
    for f in [0, 3]:
        mask = np.ones(n, bool)
        mask[starts[f]:starts[f + 1]] = False
        ntr = mask.sum()
        for i, j in idx:
            i, j = max(i, j), min(i, j)
            want = np.dot(p.X[mask, i], p.X[mask, j]) / ntr
            np.testing.assert_allclose(H[f][i, j], want, rtol=1e-12, atol=1e-15)
    # exact factors of fold 1 at two grid values: L L^T = H + lambda I
    lam = p.lam_grid[[0, 40]]
    S = B.pichol_packed_elems(d)
    Lp = gu.empty(2 * S)
    info = gu.empty(2, torch.int32)
    nb = B.pichol_potrf_workspace(1, 2)
    Hf = g["H"][S:2 * S].contiguous()
    B.pichol_potrf_shifted_batched(d, 1, Hf, 2, lam, Lp, info, gu.ws(nb), nb)
    L = gu.unpack(Lp, d, 2)
    assert np.all(info.cpu().numpy() == 0)
    for s in range(2):
        for i, j in idx:
            i, j = max(i, j), min(i, j)
            lhs = np.dot(L[s][i, :j + 1], L[s][j, :j + 1])
            rhs = H[1][i, j] + (lam[s] if i == j else 0.0)
            assert abs(lhs - rhs) <= 1e-12 * (abs(H[1][i, i]) + lam[s])


# ---------------------------------------------------------------- many problems

@pytest.fixture(scope="module")
def manyprob(gpu):
    import gpu_util
    probs = workloads.batch_problems()
    run = gpu_util.BatchRun(probs, "interp", want_W=False)
    return gpu_util, probs, run, run.run()


def test_batch_fullsize_buckets_and_status(manyprob):
    gu, probs, run, got = manyprob
    assert len(probs) == 48
    shapes = {(p.d, p.c) for p in probs}
    assert gu.B.pichol_batch_buckets(run.batch, run.method) == len(shapes)
    for i, o in enumerate(got):
        assert np.all(o["info"] == 0) and np.all(o["flags"] == 0), i
        assert np.all(np.isfinite(o["mse"])) and np.all(o["mse"] > 0), i


def test_batch_fullsize_matches_oracle_and_single(manyprob):
    gu, probs, run, got = manyprob
    order = sorted(range(len(probs)), key=lambda i: (probs[i].d, i))
    for i in order[:2]:  # the two smallest problems against the oracle
        p = probs[i]
        want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
        np.testing.assert_allclose(got[i]["mse"], want["mse"], rtol=1e-10, atol=0)
    seen = set()
    for i in range(len(probs)):  # one problem of every d against its own run
        if probs[i].d in seen:
            continue
        seen.add(probs[i].d)
        one = gu.cv(probs[i], "interp", want_W=False)
        np.testing.assert_allclose(got[i]["mse"], one["mse"], rtol=1e-13, atol=0)


# ---------------------------------------------------------------- d=2048 random features

@pytest.fixture(scope="module")
def c2(gpu):
    import gpu_util
    return gpu_util, workloads.named("rff_n20000_d2048")


def test_rff_d2048_interp_all_grid_values_match_oracle(c2):
    """The d = 2048 random-feature workload (n = 20000, k = 5, g = 6, r = 2,
    q = 64) end to end: every fold at all 64 grid values against the
    oracle's piCholesky path, weights included."""
    gu, p = c2
    got = gu.cv(p, "interp")
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    for f in range(p.k):
        H, Bm, Xv, Yv = _fold_grams(p, f)
        want = oracle.fold_interp(H, Bm, Xv, Yv, p.lam_s, p.lam_grid, p.r, want_W=True)
        assert np.all(want["info"] == 0) and np.all(want["flags"] == 0)
        np.testing.assert_allclose(got["mse"][f], want["mse"], rtol=1e-10, atol=0)
        scale = np.abs(want["W"]).max()
        assert np.abs(got["W"][f] - want["W"]).max() <= 1e-9 * scale, f


def test_rff_d2048_exact_all_grid_values_match_oracle(c2):
    """The same workload's exact CV at all 64 grid values of folds 0 and 4
    against the oracle's exact path."""
    gu, p = c2
    got = gu.cv(p, "exact", want_W=False)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    for f in [0, 4]:
        H, Bm, Xv, Yv = _fold_grams(p, f)
        want = oracle.fold_exact(H, Bm, Xv, Yv, p.lam_grid)
        assert np.all(want["info"] == 0) and np.all(want["flags"] == 0)
        np.testing.assert_allclose(got["mse"][f], want["mse"], rtol=1e-10, atol=0)


# ---------------------------------------------------------------- derivative at d=2048

@pytest.fixture(scope="module")
def c5(gpu):
    import gpu_util
    return gpu_util, workloads.named("rff_n20000_d2048")


def _grad(gu, prob, lam_grid, method="interp"):
    from test_gpu_grad import gpu_grad
    return gpu_grad(gu, prob, method, lam_grid)


def test_fullsize_grad_sampled_against_oracle(c5):
    """d = 2048 random Fourier features (n = 20000, k = 5, g = 6, r = 2):
    the derivative at four of the 64 grid values against the oracle."""
    gu, p = c5
    lam = p.lam_grid[[0, 21, 42, 63]]
    got = _grad(gu, p, lam)
    want = oracle.cv_grad(p.X, p.Y, p.k, lam, p.lam_s, p.r)
    assert np.all(got["flags"] == 0) and np.all(want["flags"] == 0)
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=1e-10, atol=0)
    assert np.abs(got["dlog"] - want["dlog"]).max() <= 1e-9 * np.abs(want["dlog"]).max()


def test_fullsize_grad_matches_central_differences(c5):
    gu, p = c5
    got = _grad(gu, p, p.lam_grid)
    h = 1e-4
    up = gu.cv(p, "interp", lam_grid=p.lam_grid * np.exp(h), want_W=False)["mse"]
    dn = gu.cv(p, "interp", lam_grid=p.lam_grid * np.exp(-h), want_W=False)["mse"]
    fd = (up - dn) / (2 * h)
    assert np.abs(fd - got["dlog"]).max() <= 1e-6 * np.abs(got["dlog"]).max()
