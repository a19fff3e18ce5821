"""The mixed-precision factorization (PICHOL_PREC_MIXED): the trailing
updates of the blocked Cholesky take their products on FP32 MFMA.

There is no FP32 oracle: the FP64 oracle is the reference and the checks are
the error bounds the arithmetic implies.

Backward error.  Each delayed update adds a sum of at most 256 products of
factor entries rounded to FP32 (relative error u = 2^-24 each) accumulated
in FP32, so the computed factor satisfies L L^T = A + E with
|E_ij| <= (2u + gamma_256) * sum_p |L_ip||L_jp| ~= 1.54e-5 * (|L||L|^T)_ij,
gamma_m = m u / (1 - m u); the FP64 parts add ~1e-13 at these sizes.  The
tests hold the ratio to 2e-5.

Forward error.  To first order the solution of (A + E) w = b differs from
the exact one by at most kappa(A) |E|_2 / |A|_2 relatively; with
|E|_2 <= 2e-5 * | |L||L|^T |_2 and | |L||L|^T |_2 a small multiple of |A|_2
for these well-conditioned inputs, hold-out errors and weights are held to
8e-5 * kappa (interpolated path: times the largest 1-norm of the fit's
evaluation weights, which bounds how far the factor errors at the samples
are amplified at a grid value).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
BACKWARD = 2e-5


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


def spd(d, seed, cond):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    ev = np.logspace(0, -np.log10(cond), d)
    return (Q * ev) @ Q.T


def factor(gu, H, lam, precision):
    nmat, d = H.shape[0], H.shape[1]
    S = gu.B.pichol_packed_elems(d)
    L = gu.empty(nmat * len(lam) * S)
    info = gu.empty(nmat * len(lam), torch.int32)
    nb = gu.B.pichol_potrf_workspace(nmat, len(lam))
    gu.B.pichol_potrf_shifted_batched(d, nmat, gu.pack(H, d), len(lam), lam, L, info,
                                      gu.ws(nb), nb, precision)
    torch.cuda.synchronize()
    return L, info.cpu().numpy()


def test_gamma_bound_constant():
    g256 = 256 * U32 / (1 - 256 * U32)
    assert 2 * U32 + g256 < BACKWARD


@pytest.mark.parametrize("d", [129, 384, 777])
def test_mixed_factor_backward_error(gu, d):
    lam = np.array([1e-3, 0.3])
    H = np.stack([spd(d, 5 * d + m, cond=1e4) for m in range(2)])
    Lm, info = factor(gu, H, lam, gu.B.PICHOL_PREC_MIXED)
    L64, info64 = factor(gu, H, lam, gu.B.PICHOL_PREC_FP64)
    assert np.all(info == 0) and np.all(info64 == 0)
    Lg = gu.unpack(Lm, d, 2 * len(lam))
    L6 = gu.unpack(L64, d, 2 * len(lam))
    worst = 0.0
    for m in range(2):
        for s, l in enumerate(lam):
            Lx = Lg[m * len(lam) + s]
            assert np.all(np.triu(Lx, 1) == 0.0) and np.all(np.diag(Lx) > 0)
            A = H[m] + l * np.eye(d)
            E = Lx @ Lx.T - A
            M = np.abs(Lx) @ np.abs(Lx).T
            ratio = np.max(np.abs(E) / M)
            worst = max(worst, ratio)
            assert ratio <= BACKWARD, f"m={m} s={s}: backward ratio {ratio:.3e}"
    print(f"d={d}: worst backward ratio {worst:.3e}")
    if d > 256:  # some trailing update ran in FP32: the factors differ
        assert np.max(np.abs(Lg - L6)) > 0.0


def test_mixed_large_batch_matches_small_batch(gu):
    """Batches of 128 or more matrices take the mixed schedule with the
    diagonal tiles in their own launches; smaller ones factor them inside
    the column updates.  The arithmetic is the same, so each matrix's factor
    must be the same bit for bit."""
    d = 300
    H = spd(d, 5 * d, cond=1e3)[None]
    lam = np.logspace(-3, 0, 128)
    Lbig, info_big = factor(gu, H, lam, gu.B.PICHOL_PREC_MIXED)
    Lsmall, info_small = factor(gu, H, lam[:8], gu.B.PICHOL_PREC_MIXED)
    assert np.all(info_big == 0) and np.all(info_small == 0)
    S = gu.B.pichol_packed_elems(d)
    np.testing.assert_array_equal(Lbig[:8 * S].cpu().numpy(), Lsmall.cpu().numpy())


def test_mixed_factor_padding_is_exact(gu):
    d = 300
    Lm, info = factor(gu, spd(d, 9, 1e2)[None], np.array([0.1]), gu.B.PICHOL_PREC_MIXED)
    assert info[0] == 0
    P = Lm.cpu().numpy().reshape(-1, 128, 128)
    last = P[5].T  # tile (2,2), column-major storage
    pad = d - 256
    np.testing.assert_array_equal(last[pad:, pad:], np.eye(128 - pad))
    assert np.all(last[pad:, :pad] == 0.0)
    for t in (3, 4):  # tiles (2,0), (2,1): padding rows are zero
        assert np.all(P[t].T[pad:, :] == 0.0)


def test_mixed_reports_non_pd(gu):
    d = 400
    H = spd(d, 4, 1e2)
    H[350, 350] = -5.0  # leading minor of order 351 is indefinite
    Lm, info = factor(gu, H[None], np.array([0.0]), gu.B.PICHOL_PREC_MIXED)
    assert 0 < info[0] <= 351


def kappa_max(prob, lam):
    starts = np.concatenate([[0], np.cumsum(
        [len(a) for a in np.array_split(np.arange(prob.n), prob.k)])])
    worst = 0.0
    for f in range(prob.k):
        mask = np.ones(prob.n, bool)
        mask[starts[f]:starts[f + 1]] = False
        Xt = prob.X[mask]
        ev = np.linalg.eigvalsh(Xt.T @ Xt / Xt.shape[0])
        worst = max(worst, (ev[-1] + lam) / (ev[0] + lam))
    return worst


def lebesgue(lam_s, lam_grid, r):
    tau_s = lam_s / np.max(lam_s)
    tau_t = lam_grid / np.max(lam_s)
    V = np.vander(tau_s, r + 1, increasing=True)
    P = np.linalg.pinv(V)
    Phi = np.vander(tau_t, r + 1, increasing=True)
    return np.max(np.sum(np.abs(Phi @ P), axis=1))


@pytest.mark.parametrize("method", ["interp", "exact"])
@pytest.mark.parametrize("n,d,c,g,q", [(1500, 520, 5, 5, 12),
                                       # q c = 640: solve launches of
                                       # 512 and more workgroups
                                       (6000, 1024, 10, 6, 64),
                                       # past the second-stream threshold
                                       (3407, 1700, 3, 4, 8)])
def test_mixed_cv_close_to_fp64_oracle(gu, method, n, d, c, g, q):
    prob = workloads.gaussian_problem(n, d, c, seed=3, g=g, r=2, q=q)
    got = gu.cv(prob, method, precision=gu.B.PICHOL_PREC_MIXED)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    if method == "interp":
        want = oracle.cv_interp(prob.X, prob.Y, prob.k, prob.lam_s, prob.lam_grid, prob.r,
                                 want_W=True)
        amp = lebesgue(prob.lam_s, prob.lam_grid, prob.r)
    else:
        want = oracle.cv_exact(prob.X, prob.Y, prob.k, prob.lam_grid, want_W=True)
        amp = 1.0
    kap = kappa_max(prob, float(np.min(prob.lam_grid)))
    tol = 4 * BACKWARD * kap * amp
    rel = np.max(np.abs(got["mse"] - want["mse"]) / want["mse"])
    wrel = np.max(np.abs(got["W"] - want["W"])) / np.max(np.abs(want["W"]))
    print(f"{method}: kappa {kap:.1f} amp {amp:.2f} tol {tol:.2e} mse rel {rel:.2e} "
          f"W rel {wrel:.2e}")
    assert rel <= tol and wrel <= tol
    # the FP64 path on the same inputs stays at the FP64 bar
    g64 = gu.cv(prob, method, precision=gu.B.PICHOL_PREC_FP64)
    np.testing.assert_allclose(g64["mse"], want["mse"], rtol=1e-10, atol=0)
