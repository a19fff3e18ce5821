"""The paper's other procedures on the GPU path: PINRMSE
(pichol_cv_pinrmse) and the multi-level Cholesky search (MChol driver over
pichol_cv_exact), against the oracle's versions.

PINRMSE tolerance: the oracle fits through Algorithm 1's normal equations,
which lose accuracy as cond(V)^2 eps, while the library applies V^+ from a
Householder QR; the curve is held to max(1e-9, 10 cond(V)^2 eps) of its
largest value (1.2e-11 for g=5, r=2 over five decades; 5e-4 for the
interpolating g=4, r=3 case, whose cond(V) is 4.8e5)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


@pytest.mark.parametrize("n,d,c,g,r,q", [(900, 300, 3, 5, 2, 17), (600, 129, 1, 4, 3, 9)])
def test_pinrmse_matches_oracle(gu, n, d, c, g, r, q):
    from paper_1404_0466_amd import variants
    p = workloads.gaussian_problem(n, d, c, seed=d, g=g, r=r, q=q)
    got = variants.pinrmse(gu.dev(p.X), gu.dev(p.Y), p.k, p.lam_s, p.lam_grid, p.r)
    want = oracle.pinrmse(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    np.testing.assert_allclose(got["mse_samples"], want["mse_samples"], rtol=1e-10, atol=0)
    tau = p.lam_s / p.lam_ref
    cond = np.linalg.cond(np.vander(tau, p.r + 1, increasing=True))
    tol = max(1e-9, 10 * cond ** 2 * np.finfo(float).eps)
    scale = np.abs(want["mse"]).max()
    assert np.abs(got["mse"] - want["mse"]).max() <= tol * scale


def test_mchol_matches_oracle(gu):
    from paper_1404_0466_amd import variants
    p = workloads.gaussian_problem(1000, 260, 3, seed=5)
    c0 = float(np.log10(p.scale)) - 1.5
    got = variants.mchol(gu.dev(p.X), gu.dev(p.Y), p.k, c0)
    want = oracle.mchol(p.X, p.Y, p.k, c0)
    assert len(got["trace"]) == len(want["trace"]) == 10
    for (gl, gv), (wl, wv) in zip(got["trace"], want["trace"]):
        np.testing.assert_array_equal(gl, wl)
        np.testing.assert_allclose(gv, wv, rtol=1e-10, atol=0)
    assert got["lam"] == want["lam"]
    assert got["factorizations"] == 10 * 3 * p.k
