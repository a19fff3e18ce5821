"""GPU accuracy diagnostics against the oracle: the NRMSE of fitted factors
against exact ones (the paper's NRMSE section) and the hold-out NRMSE."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


def _gpu_nrmse(gu, Lhat, L, d):
    """Host lower factors (m, d, d) -> GPU NRMSE per pair."""
    B = gu.B
    m = L.shape[0]
    out = gu.empty(m)
    nb = B.pichol_factor_nrmse_workspace(d, m)
    B.pichol_factor_nrmse(d, m, gu.pack(Lhat, d), gu.pack(L, d), out, gu.ws(nb), nb)
    gu.torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("d", [1, 127, 300])
def test_factor_nrmse_matches_oracle(gu, d):
    """Ragged orders (padding excluded) and several tiles: the GPU reduction
    equals the oracle's definition; the mean predictor gives 1."""
    rng = np.random.default_rng(40 + d)
    L = np.stack([np.tril(rng.standard_normal((d, d))) for _ in range(3)])
    Lhat = L + 1e-3 * np.stack([np.tril(rng.standard_normal((d, d))) for _ in range(3)])
    il = np.tril_indices(d)
    mean = np.stack([np.tril(np.full((d, d), x[il].mean())) for x in L])
    got = _gpu_nrmse(gu, np.concatenate([Lhat, mean]), np.concatenate([L, L]), d)
    want = [oracle.factor_nrmse(a, b) for a, b in zip(np.concatenate([Lhat, mean]),
                                                       np.concatenate([L, L]))]
    np.testing.assert_allclose(got, want, rtol=1e-12)  # NaN where both are 0/0
    if d > 1:  # a 1 x 1 factor has no spread about its mean: 0/0
        np.testing.assert_allclose(got[3:], 1.0, rtol=1e-12)
    else:
        assert np.all(np.isnan(got[3:]))


def test_factor_nrmse_of_interpolated_factors(gu):
    """End to end on one fold: GPU interpolated factors (pichol_eval) against
    GPU exact factors (pichol_potrf_shifted_batched), compared with the same
    measure on the oracle's fit and factors."""
    B = gu.B
    p = workloads.rff_problem(1200, 260, 10, seed=8, g=5, q=7)
    d, g = p.d, len(p.lam_s)
    lam_ref = float(np.max(p.lam_s))
    H, _ = oracle.fold_gram(p.X, p.Y, p.k, 0)[:2]
    # GPU: factors at the samples, fit, evaluation at the grid, exact factors
    Hd = gu.pack(H[None], d)
    S = B.pichol_packed_elems(d)
    Ls = gu.empty(g * S)
    info = gu.empty(g, gu.torch.int32)
    nbw = B.pichol_potrf_workspace(1, g)
    B.pichol_potrf_shifted_batched(d, 1, Hd, g, p.lam_s, Ls, info, gu.ws(nbw), nbw)
    th, tht = gu.empty(3 * S), gu.empty(3 * S)
    B.pichol_fit(d, 1, g, p.r, p.lam_s, lam_ref, Ls, th, tht)
    q = len(p.lam_grid)
    Lhat = gu.empty(q * S)
    nbe = B.pichol_lambda_workspace(q)
    B.pichol_eval(d, 1, p.r, th, q, p.lam_grid, lam_ref, Lhat, gu.ws(nbe), nbe)
    Lex = gu.empty(q * S)
    infoq = gu.empty(q, gu.torch.int32)
    nbq = B.pichol_potrf_workspace(1, q)
    B.pichol_potrf_shifted_batched(d, 1, Hd, q, p.lam_grid, Lex, infoq, gu.ws(nbq), nbq)
    out = gu.empty(q)
    nbn = B.pichol_factor_nrmse_workspace(d, q)
    B.pichol_factor_nrmse(d, q, Lhat, Lex, out, gu.ws(nbn), nbn)
    gu.torch.cuda.synchronize()
    got = out.cpu().numpy()
    # oracle: Algorithm 1 steps 1-6, the evaluation and the exact factors
    T = np.stack([oracle.pack_lower(oracle.cholesky(H, lam)[0]) for lam in p.lam_s])
    Th = oracle.fit(T, p.lam_s, p.r, lam_ref)
    want = [oracle.factor_nrmse(oracle.unpack_lower(oracle.evaluate(Th, lam, lam_ref), d),
                                oracle.cholesky(H, lam)[0]) for lam in p.lam_grid]
    np.testing.assert_allclose(got, want, rtol=1e-8, atol=1e-13)
    assert np.all(got < 1.0)


def test_holdout_nrmse_matches_oracle(gu):
    B = gu.B
    p = workloads.rff_problem(1500, 200, 10, seed=9, g=5, q=9)
    got_cv = gu.cv(p, "interp", want_W=False)
    n, d = p.X.shape
    c = p.Y.shape[1]
    q = len(p.lam_grid)
    prob = B.make_problem(n, d, c, p.k, len(p.lam_s), p.r, q, True)
    err = gu.dev(got_cv["mse"].reshape(-1))
    nr = gu.empty(p.k * q)
    B.pichol_holdout_nrmse(prob, gu.dev(p.Y), err, nr)
    gu.torch.cuda.synchronize()
    got = nr.cpu().numpy().reshape(p.k, q)
    want = oracle.cv_nrmse(p.Y, p.k, oracle.cv_interp(p.X, p.Y, p.k, p.lam_s,
                                                      p.lam_grid, p.r)["sse"])
    np.testing.assert_allclose(got, want, rtol=1e-9)


def test_nrmse_argument_errors(gu):
    B = gu.B
    with pytest.raises(B.PicholError) as e:
        B.pichol_factor_nrmse(0, 1, gu.empty(1), gu.empty(1), gu.empty(1), gu.ws(256), 256)
    assert e.value.status == B.PICHOL_ERR_ARG
    nb = B.pichol_factor_nrmse_workspace(300, 2)
    with pytest.raises(B.PicholError) as e:
        S = B.pichol_packed_elems(300)
        B.pichol_factor_nrmse(300, 2, gu.empty(2 * S), gu.empty(2 * S), gu.empty(2),
                              gu.ws(nb - 8), nb - 8)
    assert e.value.status == B.PICHOL_ERR_WORKSPACE
