"""Vectorisations of a factor (Sec. 5) for the layout comparison:
pichol_vectorize against the oracle's orders (bit for bit: pure data
movement), and the flat fit / evaluation against the oracle's fit and
evaluation (Algorithm 1 on any vectorisation, entry by entry)."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


def rand_lower(d, nmat, seed):
    rng = np.random.default_rng(seed)
    return np.tril(rng.standard_normal((nmat, d, d)))


@pytest.mark.parametrize("d", [5, 128, 200, 384])
def test_vectorize_rowwise_and_full(gu, d):
    B = gu.B
    L = rand_lower(d, 2, d)
    P = gu.pack(L, d)
    for layout in [B.PICHOL_LAYOUT_ROWWISE, B.PICHOL_LAYOUT_FULL]:
        N = B.pichol_vector_length(d, layout)
        T = torch.zeros(2 * N, dtype=torch.float64, device="cuda:0")
        B.pichol_vectorize(d, 2, P, layout, 1, T)
        got = T.cpu().numpy().reshape(2, N)
        for m in range(2):
            if layout == B.PICHOL_LAYOUT_ROWWISE:
                want = oracle.pack_lower(L[m])
            else:
                want = L[m].reshape(-1)
            np.testing.assert_array_equal(got[m, :want.size], want)


@pytest.mark.parametrize("d,h0", [(256, 128), (300, 64), (129, 16), (64, 128)])
def test_vectorize_recursive(gu, d, h0):
    B = gu.B
    L = rand_lower(d, 1, d + h0)
    N = B.pichol_vector_length(d, B.PICHOL_LAYOUT_RECURSIVE)
    T = torch.zeros(N, dtype=torch.float64, device="cuda:0")
    B.pichol_vectorize(d, 1, gu.pack(L, d), B.PICHOL_LAYOUT_RECURSIVE, h0, T)
    order = oracle.recursive_order(d, h0)
    want = np.array([L[0][i, j] for i, j in order])
    np.testing.assert_array_equal(T.cpu().numpy()[:want.size], want)


def test_fit_and_eval_on_vectors(gu):
    B = gu.B
    rng = np.random.default_rng(5)
    g, r, N, q = 5, 2, 4096, 7
    lam_s = np.logspace(-3, 0, g)
    lam_ref = lam_s.max()
    T = rng.standard_normal((g, N))
    theta = gu.empty(3 * N)
    B.pichol_fit_vec(N, 1, g, r, lam_s, lam_ref, gu.dev(T.reshape(-1)), theta)
    want = oracle.fit(T, lam_s, r, lam_ref)
    got = theta.cpu().numpy().reshape(3, N)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11 * np.abs(want).max())
    lam = np.logspace(-3, 0, q)
    out = gu.empty(q * N)
    nb = B.pichol_lambda_workspace(q)
    B.pichol_eval_vec(N, 1, r, theta, q, lam, lam_ref, out, gu.ws(nb), nb)
    got = out.cpu().numpy().reshape(q, N)
    for t in range(q):
        w = oracle.evaluate(want, lam[t], lam_ref)
        np.testing.assert_allclose(got[t], w, rtol=0, atol=1e-11 * np.abs(w).max())
