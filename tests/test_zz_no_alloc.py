"""pichol_holdout_noalloc, the hold-out step for callers that cannot
allocate: its partial sums live in the library's static device scratch
instead of a workspace.  Checked through the C-ABI against pichol_holdout
(same kernels, so bit for bit) and against the oracle's direct residual, on
two calls in a row, the second with a smaller problem, so that a stale or
misaddressed scratch would show."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


def _case(gu, n, d, c, k, q, seed):
    B = gu.B
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((n, c))
    W = rng.standard_normal((k, q, d, c)) / np.sqrt(d)
    dp = B.pichol_padded_order(d)
    ldz = B.pichol_slab_cols(q, c)
    Z = np.zeros((k, dp, ldz))
    for m in range(k):
        for t in range(q):
            Z[m, :d, t * c:(t + 1) * c] = W[m, t]
    gr = gu.gram(X, Y, k)
    nv = gu.fold_sizes(n, k)
    return X, Y, W, gu.dev(Z), gr, nv


def _run_both(gu, d, c, k, q, Zd, gr, nv):
    B = gu.B
    nb = B.pichol_holdout_workspace(d, k, q, c)
    assert nb <= B.PICHOL_HOLDOUT_SCRATCH_BYTES
    e_ws, f_ws = gu.empty(k * q), gu.empty(k * q, torch.int32)
    f_ws.zero_()
    B.pichol_holdout(d, k, c, q, Zd, gr["G"], gr["C"], gr["yy"], nv, e_ws, f_ws,
                     gu.ws(nb), nb)
    e_na, f_na = gu.empty(k * q), gu.empty(k * q, torch.int32)
    e_na.fill_(float("nan"))
    f_na.zero_()
    B.pichol_holdout_noalloc(d, k, c, q, Zd, gr["G"], gr["C"], gr["yy"], nv, e_na,
                             f_na)
    torch.cuda.synchronize()
    return (e_ws.cpu().numpy().reshape(k, q), f_ws.cpu().numpy().reshape(k, q),
            e_na.cpu().numpy().reshape(k, q), f_na.cpu().numpy().reshape(k, q))


def test_noalloc_matches_workspace_call_twice(gu):
    cases = [(2000, 300, 10, 5, 31, 1), (600, 129, 3, 3, 5, 2)]  # second smaller
    for n, d, c, k, q, seed in cases:
        X, Y, W, Zd, gr, nv = _case(gu, n, d, c, k, q, seed)
        e_ws, f_ws, e_na, f_na = _run_both(gu, d, c, k, q, Zd, gr, nv)
        np.testing.assert_array_equal(e_na, e_ws)
        np.testing.assert_array_equal(f_na, f_ws)
        assert np.all(f_na == 0)
        b = oracle.fold_bounds(n, k)
        for m in range(k):
            Xv, Yv = X[b[m]:b[m + 1]], Y[b[m]:b[m + 1]]
            for t in range(q):
                want = oracle.holdout_sse(Xv, Yv, W[m, t]) / (Xv.shape[0] * c)
                assert abs(e_na[m, t] - want) <= 1e-10 * want, (n, m, t)


def test_noalloc_rejects_sizes_beyond_the_scratch(gu):
    B = gu.B
    # d = 4096, q = 64, c = 10: 13 folds need 17 MB of partial sums
    d, k, c, q = 4096, 13, 10, 64
    assert B.pichol_holdout_workspace(d, k, q, c) > B.PICHOL_HOLDOUT_SCRATCH_BYTES
    one = gu.empty(1)
    flags = gu.empty(1, torch.int32)
    with pytest.raises(B.PicholError) as e:
        B.pichol_holdout_noalloc(d, k, c, q, one, one, one, one,
                                 np.ones(k, np.int64), one, flags)
    assert e.value.status == B.PICHOL_ERR_WORKSPACE
    assert "static scratch" in str(e.value)
