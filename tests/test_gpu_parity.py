"""Parity of the HIP path with the CPU oracle, element by element, on
seeded inputs.  Every call goes through the C-ABI (``binding``).

Tolerances.  Both sides compute in IEEE FP64 but accumulate in different
orders (blocked MFMA sums on the GPU, left-to-right loops in the oracle).
For a Cholesky factor of a matrix with condition number kappa the entrywise
difference of two backward-stable FP64 factorizations is bounded by a
modest multiple of kappa * d * eps * |L|; the inputs below have kappa <= 1e4
and d <= 400, which puts the bound near 1e-9 |L| in the worst case and
observed differences far below.  The pipeline's hold-out errors are held to
the 1e-10 relative bar the method's FP64 path is specified at.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


def spd(d, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    ev = np.logspace(0, -np.log10(cond), d)
    return (Q * ev) @ Q.T


def close(a, b, rel, name=""):
    scale = max(np.max(np.abs(b)), 1e-300)
    diff = np.max(np.abs(a - b)) if a.size else 0.0
    assert np.all(np.isfinite(a)) == np.all(np.isfinite(b)), name
    assert diff <= rel * scale, f"{name}: max diff {diff:.3e} > {rel:.1e} * {scale:.3e}"


# ------------------------------------------------------------------ layout

@pytest.mark.parametrize("d", [1, 7, 127, 128, 129, 300])
def test_pack_unpack_roundtrip(gu, d):
    rng = np.random.default_rng(d)
    A = rng.standard_normal((2, d, d))
    P = gu.pack(A, d)
    L = gu.unpack(P, d, 2)
    np.testing.assert_array_equal(L, np.tril(A))


# ------------------------------------------------------------------ Gram

@pytest.mark.parametrize("n,d,c,k", [(53, 7, 3, 5), (1003, 300, 4, 5), (640, 128, 10, 4),
                                     (97, 129, 1, 3)])
def test_gram_matches_oracle(gu, n, d, c, k):
    rng = np.random.default_rng(n + d)
    X = rng.standard_normal((n, d))
    Y = np.sign(rng.standard_normal((n, c)))
    out = gu.gram(X, Y, k)
    torch.cuda.synchronize()
    H = gu.unpack(out["H"], d, k)
    dp = gu.B.pichol_padded_order(d)
    Bf = out["B"].cpu().numpy().reshape(k, dp, c)
    sizes = gu.fold_sizes(n, k)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    G = out["G"].cpu().numpy().reshape(k, dp // 128, dp // 128, 128, 128)
    C = out["C"].cpu().numpy().reshape(k, dp, c)
    yy = out["yy"].cpu().numpy()
    for f in range(k):
        Ho, Bo, _ = oracle.fold_gram(X, Y, k, f)
        close(H[f], np.tril(Ho), 1e-13, "H")
        close(Bf[f, :d], Bo, 1e-13, "B")
        assert np.all(Bf[f, d:] == 0.0)
        # validation-block Grams: X_b^T X_b as full tiles, column-major
        Xb, Yb = X[starts[f]:starts[f + 1]], Y[starts[f]:starts[f + 1]]
        Gd = G[f].transpose(0, 3, 1, 2).reshape(dp, dp)  # tile (I,J) elem (r,c) at [c][r]
        close(Gd[:d, :d], Xb.T @ Xb, 1e-13, "G")
        assert np.all(Gd[d:, :] == 0.0) and np.all(Gd[:, d:] == 0.0)
        close(C[f, :d], Xb.T @ Yb, 1e-13, "C")
        np.testing.assert_allclose(yy[f], np.sum(Yb * Yb), rtol=1e-13)


@pytest.mark.parametrize("n,d,k", [(16384, 1371, 8), (16392, 1371, 8),
                                   (24576, 1152, 12)])
def test_gram_split_last_round_matches_oracle(gu, n, d, k):
    """Gram tile counts just above one round of 512 workgroups (two per CU
    on a 256-CU MI355X), so the last tiles are summed over row chunks and
    added up by the tail kernel:
      - 8 folds of 2048 rows, d = 1371 (11 tile columns, the last one
        ragged): 8 x 66 = 528 tiles, the last 16 (among them the ragged
        diagonal tile) in eight chunks;
      - the same with folds of 2049 rows (chunks of 260 rows, the last one
        229 rows long, not a multiple of four);
      - 12 folds of 2048 rows, d = 1152: 12 x 45 = 540 tiles, the last 28
        in eight chunks, and the combine for more than eight folds.
    Every block's G and C, and H of the first and last fold, against the
    oracle's definitions."""
    c = 3
    rng = np.random.default_rng(n + d)
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((n, c))
    out = gu.gram(X, Y, k)
    torch.cuda.synchronize()
    H = gu.unpack(out["H"], d, k)
    dp = gu.B.pichol_padded_order(d)
    G = out["G"].cpu().numpy().reshape(k, dp // 128, dp // 128, 128, 128)
    C = out["C"].cpu().numpy().reshape(k, dp, c)
    starts = np.concatenate([[0], np.cumsum(gu.fold_sizes(n, k))])
    for b in range(k):
        Xb, Yb = X[starts[b]:starts[b + 1]], Y[starts[b]:starts[b + 1]]
        Gd = G[b].transpose(0, 3, 1, 2).reshape(dp, dp)
        close(Gd[:d, :d], Xb.T @ Xb, 1e-13, "G")
        assert np.all(Gd[d:, :] == 0.0) and np.all(Gd[:, d:] == 0.0)
        # the mirror of every tile below the diagonal is its exact transpose
        for I in range(dp // 128):
            for J in range(I):
                np.testing.assert_array_equal(G[b, J, I], G[b, I, J].T)
        close(C[b, :d], Xb.T @ Yb, 1e-13, "C")
    for f in (0, k - 1):
        Ho, _, _ = oracle.fold_gram(X, Y, k, f)
        close(H[f], np.tril(Ho), 1e-13, "H")
    # no atomics anywhere: a second call gives the same bits
    again = gu.gram(X, Y, k)
    torch.cuda.synchronize()
    for name in ("G", "C", "H", "B", "yy"):
        assert torch.equal(again[name], out[name]), name


# ------------------------------------------------------------------ factorization

@pytest.mark.parametrize("d", [1, 5, 127, 128, 129, 257, 384])
def test_potrf_matches_oracle(gu, d):
    nmat, lam = 2, np.array([1e-3, 0.05, 1.0])
    H = np.stack([spd(d, 10 * d + m, cond=1e3) for m in range(nmat)])
    Hp = gu.pack(H, d)
    S = gu.B.pichol_packed_elems(d)
    L = gu.empty(nmat * len(lam) * S)
    info = gu.empty(nmat * len(lam), torch.int32)
    nb = gu.B.pichol_potrf_workspace(nmat, len(lam))
    w = gu.ws(nb)
    gu.B.pichol_potrf_shifted_batched(d, nmat, Hp, len(lam), lam, L, info, w, nb)
    Lg = gu.unpack(L, d, nmat * len(lam))
    assert np.all(info.cpu().numpy() == 0)
    for m in range(nmat):
        for s, l in enumerate(lam):
            Lo, io = oracle.cholesky(H[m], l)
            assert io == 0
            close(Lg[m * len(lam) + s], Lo, 1e-11, f"L d={d} m={m} s={s}")


@pytest.mark.parametrize("group", [1, 2, 3, 8])
@pytest.mark.parametrize("d", [300, 1000])
def test_potrf_panel_groups_match_oracle(gu, d, group):
    nmat, lam = 2, np.array([1e-3, 0.4])
    H = np.stack([spd(d, 7 * d + m, cond=1e3) for m in range(nmat)])
    S = gu.B.pichol_packed_elems(d)
    L = gu.empty(nmat * len(lam) * S)
    info = gu.empty(nmat * len(lam), torch.int32)
    nb = gu.B.pichol_potrf_workspace(nmat, len(lam))
    old = gu.B.pichol_get_option(gu.B.PICHOL_OPT_PANEL_GROUP)
    gu.B.pichol_set_option(gu.B.PICHOL_OPT_PANEL_GROUP, group)
    try:
        gu.B.pichol_potrf_shifted_batched(d, nmat, gu.pack(H, d), len(lam), lam, L, info,
                                          gu.ws(nb), nb)
        Lg = gu.unpack(L, d, nmat * len(lam))
    finally:
        gu.B.pichol_set_option(gu.B.PICHOL_OPT_PANEL_GROUP, old)
    assert np.all(info.cpu().numpy() == 0)
    for m in range(nmat):
        for s, l in enumerate(lam):
            Lo, io = oracle.cholesky(H[m], l)
            close(Lg[m * len(lam) + s], Lo, 1e-11, f"L d={d} group={group}")


def test_potrf_padding_and_upper_zero(gu):
    d = 200
    H = spd(d, 3)
    S = gu.B.pichol_packed_elems(d)
    L = gu.empty(S)
    info = gu.empty(1, torch.int32)
    nb = gu.B.pichol_potrf_workspace(1, 1)
    gu.B.pichol_potrf_shifted_batched(d, 1, gu.pack(H[None], d), 1, [0.1], L, info,
                                      gu.ws(nb), nb)
    torch.cuda.synchronize()
    P = L.cpu().numpy().reshape(-1, 128, 128)  # tiles (0,0), (1,0), (1,1)
    t11 = P[2].T  # column-major storage -> [row][col]
    assert np.all(np.triu(P[0].T, 1) == 0.0) and np.all(np.triu(t11, 1) == 0.0)
    pad = d - 128
    np.testing.assert_array_equal(t11[pad:, pad:], np.eye(128 - pad))
    assert np.all(t11[pad:, :pad] == 0.0)
    assert np.all(P[1].T[pad:, :] == 0.0)


@pytest.mark.parametrize("col", [0, 130, 199])
def test_potrf_reports_first_failing_pivot(gu, col):
    d = 200
    h = np.linspace(1.0, 2.0, d)
    h[col] = -1.0
    H = np.diag(h)
    H[col, 0 if col else 1] = H[0 if col else 1, col] = 0.01
    S = gu.B.pichol_packed_elems(d)
    L = gu.empty(2 * S)
    info = gu.empty(2, torch.int32)
    nb = gu.B.pichol_potrf_workspace(1, 2)
    lam = [0.5, 2.0]
    gu.B.pichol_potrf_shifted_batched(d, 1, gu.pack(H[None], d), 2, lam, L, info,
                                      gu.ws(nb), nb)
    got = info.cpu().numpy()
    want = [oracle.cholesky(H, l)[1] for l in lam]
    assert want[0] == col + 1 and want[1] == 0
    np.testing.assert_array_equal(got, want)
    assert gu.B.pichol_check(info, 2, None, 0) == gu.B.PICHOL_ERR_NOT_PD


# ------------------------------------------------------------------ fit / evaluate

@pytest.mark.parametrize("d,g,r", [(129, 4, 2), (300, 6, 2), (64, 3, 2), (150, 5, 4)])
def test_fit_and_eval_match_oracle(gu, d, g, r):
    H = spd(d, d + g, cond=1e2)
    lam_s = np.logspace(-3, 0, g)
    lam_ref = lam_s.max()
    S = gu.B.pichol_packed_elems(d)
    L = gu.empty(g * S)
    info = gu.empty(g, torch.int32)
    nb = gu.B.pichol_potrf_workspace(1, g)
    gu.B.pichol_potrf_shifted_batched(d, 1, gu.pack(H[None], d), g, lam_s, L, info,
                                      gu.ws(nb), nb)
    th = gu.empty((r + 1) * S)
    tht = gu.empty((r + 1) * S)
    gu.B.pichol_fit(d, 1, g, r, lam_s, lam_ref, L, th, tht)
    lam_t = np.array([2e-3, 0.02, 0.3, 0.9])
    Lh = gu.empty(len(lam_t) * S)
    nb = gu.B.pichol_lambda_workspace(len(lam_t))
    gu.B.pichol_eval(d, 1, r, th, len(lam_t), lam_t, lam_ref, Lh, gu.ws(nb), nb)
    Thg = gu.unpack(th, d, r + 1)
    Lhg = gu.unpack(Lh, d, len(lam_t))
    # oracle: its own factors, Algorithm 1, evaluation
    T = np.stack([oracle.pack_lower(oracle.cholesky(H, l)[0]) for l in lam_s])
    Tho = oracle.fit(T, lam_s, r, lam_ref)
    cond = np.linalg.cond(np.vander(lam_s / lam_ref, r + 1, increasing=True))
    for j in range(r + 1):
        close(Thg[j], oracle.unpack_lower(Tho[j], d), 1e-11 * cond ** 2, f"theta{j}")
    for t, lam in enumerate(lam_t):
        Lo = oracle.unpack_lower(oracle.evaluate(Tho, lam, lam_ref), d)
        close(Lhg[t], Lo, 1e-11 * cond ** 2, f"Lhat t={t}")
    # the row-major copy holds the same planes with every tile transposed
    a = th.cpu().numpy().reshape(-1, 128, 128)
    b = tht.cpu().numpy().reshape(-1, 128, 128)
    np.testing.assert_array_equal(a, b.transpose(0, 2, 1))


# ------------------------------------------------------------------ solves

def _factors(gu, H, lam, d):
    nm = len(lam)
    S = gu.B.pichol_packed_elems(d)
    L = gu.empty(nm * S)
    info = gu.empty(nm, torch.int32)
    nb = gu.B.pichol_potrf_workspace(1, nm)
    gu.B.pichol_potrf_shifted_batched(d, 1, gu.pack(H[None], d), nm, lam, L, info,
                                      gu.ws(nb), nb)
    return L


@pytest.mark.parametrize("d,c,q", [(1, 1, 2), (100, 3, 5), (128, 10, 13), (300, 10, 31),
                                   (257, 17, 3)])
def test_solve_factors_matches_oracle(gu, d, c, q):
    rng = np.random.default_rng(d + c)
    H = spd(d, d, cond=1e3)
    lam = np.logspace(-3, 0, q)
    L = _factors(gu, H, lam, d)
    dp = gu.B.pichol_padded_order(d)
    Bh = np.zeros((dp, c))
    Bh[:d] = rng.standard_normal((d, c))
    ldz = gu.B.pichol_slab_cols(q, c)
    Z = gu.empty(dp * ldz)
    flags = gu.empty(q, torch.int32)
    gu.B.pichol_solve_factors(d, 1, q, c, L, gu.dev(Bh), Z, flags)
    Wg = gu.slab_to_w(Z, d, 1, q, c)[0]
    assert np.all(flags.cpu().numpy() == 0)
    Zh = Z.cpu().numpy().reshape(dp, ldz)
    assert np.all(Zh[d:] == 0.0) and np.all(Zh[:, q * c:] == 0.0)
    for t in range(q):
        Lo, _ = oracle.cholesky(H, lam[t])
        Wo, fo = oracle.solve(Lo, Bh[:d])
        assert fo == 0
        close(Wg[t], Wo, 1e-10, f"W t={t}")


@pytest.mark.parametrize("d,c,g,r,q", [(1, 2, 3, 2, 4), (129, 3, 4, 2, 7), (300, 10, 6, 2, 31),
                                       (256, 10, 4, 2, 64), (140, 5, 5, 4, 9)])
def test_solve_interp_matches_oracle(gu, d, c, g, r, q):
    rng = np.random.default_rng(d * q)
    H = spd(d, d + 1, cond=1e2)
    lo = -3 if r <= 2 else -1  # keep V of the quartic fit reasonably conditioned
    lam_s = np.logspace(lo, 0, g)
    lam_ref = lam_s.max()
    lam = np.logspace(lo, 0, q)
    # the oracle solves Algorithm 1's normal equations, accurate to about
    # cond(V)^2 eps; the library's QR fit to cond(V) eps
    cond = np.linalg.cond(np.vander(lam_s / lam_ref, r + 1, increasing=True))
    rel = max(1e-9, 10 * cond ** 2 * EPS * 1e2)
    L = _factors(gu, H, lam_s, d)
    S = gu.B.pichol_packed_elems(d)
    th = gu.empty((r + 1) * S)
    tht = gu.empty((r + 1) * S)
    gu.B.pichol_fit(d, 1, g, r, lam_s, lam_ref, L, th, tht)
    dp = gu.B.pichol_padded_order(d)
    Bh = np.zeros((dp, c))
    Bh[:d] = rng.standard_normal((d, c))
    ldz = gu.B.pichol_slab_cols(q, c)
    Z = gu.empty(dp * ldz)
    flags = gu.empty(q, torch.int32)
    nb = gu.B.pichol_solve_interp_workspace(d, 1, q, c)
    gu.B.pichol_solve_interp(d, 1, c, r, th, tht, gu.dev(Bh), q, lam, lam_ref, Z,
                             flags, gu.ws(nb), nb)
    Wg = gu.slab_to_w(Z, d, 1, q, c)[0]
    T = np.stack([oracle.pack_lower(oracle.cholesky(H, l)[0]) for l in lam_s])
    Tho = oracle.fit(T, lam_s, r, lam_ref)
    fl = flags.cpu().numpy()
    for t in range(q):
        Lo = oracle.unpack_lower(oracle.evaluate(Tho, lam[t], lam_ref), d)
        Wo, fo = oracle.solve(Lo, Bh[:d])
        assert fl[t] == fo
        close(Wg[t], Wo, rel, f"W t={t}")


def _library_fit_solve(H, lam_s, lam_ref, r, lam, Bd):
    import gpu_util
    return gpu_util.library_fit_solve(H, lam_s, lam_ref, r, lam, Bd)


@pytest.mark.parametrize("d,c,g,r,q", [(140, 5, 5, 4, 9), (140, 5, 6, 4, 9),
                                       (200, 3, 6, 3, 12), (257, 10, 6, 4, 17)])
def test_solve_interp_high_degree_wide_range(gu, d, c, g, r, q):
    """Degrees 3 and 4 over three decades (tau in [1e-3, 1], cond(V) up to
    2.6e5): the oracle's normal equations are good only to cond(V)^2 eps
    there, so the HIP path (whose fit multiplies by a pseudo-inverse from a
    Householder QR) is held at 1e-10 to the same steps composed from LAPACK
    routines, which two backward-stable fits meet to about 3e-12."""
    rng = np.random.default_rng(7 * d + q)
    H = spd(d, d + 3, cond=1e2)
    lam_s = np.logspace(-3, 0, g)
    lam_ref = lam_s.max()
    lam = np.logspace(-3, 0, q)
    L = _factors(gu, H, lam_s, d)
    S = gu.B.pichol_packed_elems(d)
    th = gu.empty((r + 1) * S)
    tht = gu.empty((r + 1) * S)
    gu.B.pichol_fit(d, 1, g, r, lam_s, lam_ref, L, th, tht)
    dp = gu.B.pichol_padded_order(d)
    Bh = np.zeros((dp, c))
    Bh[:d] = rng.standard_normal((d, c))
    ldz = gu.B.pichol_slab_cols(q, c)
    Z = gu.empty(dp * ldz)
    flags = gu.empty(q, torch.int32)
    nb = gu.B.pichol_solve_interp_workspace(d, 1, q, c)
    gu.B.pichol_solve_interp(d, 1, c, r, th, tht, gu.dev(Bh), q, lam, lam_ref, Z,
                             flags, gu.ws(nb), nb)
    Wg = gu.slab_to_w(Z, d, 1, q, c)[0]
    assert np.all(flags.cpu().numpy() == 0)
    want = _library_fit_solve(H, lam_s, lam_ref, r, lam, Bh[:d])
    for t in range(q):
        close(Wg[t], want[t], 1e-10, f"W t={t}")


def test_cv_interp_quartic_wide_range_matches_library_composition(gu):
    """The whole interpolated pipeline at degree 4 (g = 6) over four decades
    of lambda, hold-out errors at 1e-10 against the library composition of
    the same steps (validation residual formed directly)."""
    p = workloads.gaussian_problem(1200, 160, 4, seed=17, k=3, g=6, q=13,
                                   lam_range=(1e-4, 1.0))
    lam_s = p.lam_grid[[0, 3, 5, 7, 9, 12]]
    got = gu.cv(p, "interp", lam_s=lam_s, r=4)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    b = oracle.fold_bounds(p.n, p.k)
    lam_ref = lam_s.max()
    for f in range(p.k):
        mask = np.ones(p.n, bool)
        mask[b[f]:b[f + 1]] = False
        Xt, Yt, Xv, Yv = p.X[mask], p.Y[mask], p.X[~mask], p.Y[~mask]
        ntr = mask.sum()
        H, Bm = Xt.T @ Xt / ntr, Xt.T @ Yt / ntr
        W = _library_fit_solve(H, lam_s, lam_ref, 4, p.lam_grid, Bm)
        for t in range(len(p.lam_grid)):
            close(got["W"][f, t], W[t], 1e-10, f"W f={f} t={t}")
            mse = np.sum((Yv - Xv @ W[t]) ** 2) / Yv.size
            assert abs(got["mse"][f, t] - mse) <= 1e-10 * mse, (f, t)


@pytest.mark.parametrize("d,c,g,r,q", [(1, 2, 3, 2, 4), (129, 17, 4, 2, 7),
                                       (300, 10, 6, 2, 31), (257, 1, 5, 4, 9),
                                       (384, 33, 3, 0, 5), (200, 16, 7, 6, 3)])
def test_solve_forms_agree(gu, d, c, g, r, q):
    """The two forms of the interpolated solves (per lambda with the
    diagonal blocks fused into the steps, and stacked over the planes) on
    ragged shapes: c above and at 16, one tile, degrees 0 to 6 (the generic
    plane count), q*c not a multiple of the units per workgroup."""
    B = gu.B
    rng = np.random.default_rng(3 * d + c)
    H = spd(d, d + 7, cond=1e2)
    lam_s = np.logspace(-2, 0, g)
    lam_ref = lam_s.max()
    lam = np.logspace(-2, 0, q)
    L = _factors(gu, H, lam_s, d)
    S = B.pichol_packed_elems(d)
    th = gu.empty((r + 1) * S)
    tht = gu.empty((r + 1) * S)
    B.pichol_fit(d, 1, g, r, lam_s, lam_ref, L, th, tht)
    dp = B.pichol_padded_order(d)
    Bh = np.zeros((dp, c))
    Bh[:d] = rng.standard_normal((d, c))
    ldz = B.pichol_slab_cols(q, c)
    nb = B.pichol_solve_interp_workspace(d, 1, q, c)
    out = {}
    try:
        for form in (2, 1):
            B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, form)
            Z = gu.empty(dp * ldz)
            flags = gu.empty(q, torch.int32)
            B.pichol_solve_interp(d, 1, c, r, th, tht, gu.dev(Bh), q, lam, lam_ref, Z,
                                  flags, gu.ws(nb), nb)
            torch.cuda.synchronize()
            out[form] = (Z.cpu().numpy().reshape(dp, ldz), flags.cpu().numpy())
    finally:
        B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, 0)
    Z0, f0 = out[2]
    Z1, f1 = out[1]
    np.testing.assert_array_equal(f0, f1)
    assert np.all(Z0[d:] == 0.0) and np.all(Z0[:, q * c:] == 0.0)
    close(Z0[:d, :q * c], Z1[:d, :q * c], 1e-12, "forms")


@pytest.mark.parametrize("form,c", [(1, 10), (2, 10), (1, 1), (2, 1), (0, 1)])
def test_cv_solve_forms_match_oracle(gu, form, c):
    """Each form of the solves, selected by option (0: the automatic choice,
    stacked for c = 1), against the oracle on the Gaussian workload."""
    B = gu.B
    p = workloads.gaussian_problem(2000, 256, c, seed=0, g=4, r=2, q=31)
    B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, form)
    try:
        got = gu.cv(p, "interp")
    finally:
        B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, 0)
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True)
    _check_cv(got, want)


# ------------------------------------------------------------------ pipelines

def _check_cv(got, want, rel_err=1e-10, rel_w=1e-9):
    np.testing.assert_array_equal(got["info"], want["info"])
    np.testing.assert_array_equal(got["flags"], want["flags"])
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=rel_err, atol=0)
    if want.get("W") is not None:
        close(got["W"], want["W"], rel_w, "W")


def test_cv_interp_gauss_n2000_d256(gu):
    p = workloads.named("gauss_n2000_d256")
    got = gu.cv(p, "interp")
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True)
    _check_cv(got, want)


def test_cv_exact_gauss_n2000_d256(gu):
    p = workloads.named("gauss_n2000_d256")
    got = gu.cv(p, "exact")
    want = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid, want_W=True)
    _check_cv(got, want)


@pytest.mark.parametrize("method", ["interp", "exact"])
def test_cv_ragged(gu, method):
    """Ragged everywhere: n not divisible by k, d not a multiple of the tile,
    q*c not a multiple of 128, c > 16 on the exact path."""
    p = workloads.gaussian_problem(1003, 300, 3, seed=11, g=5, q=13)
    if method == "interp":
        got = gu.cv(p, "interp")
        want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True)
    else:
        p = workloads.gaussian_problem(700, 150, 18, seed=12, q=5)
        got = gu.cv(p, "exact")
        want = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid, want_W=True)
    _check_cv(got, want)


def test_cv_rff_midsize(gu):
    """Random-Fourier-feature workload (the structure of the benchmark's
    data) at a size the oracle finishes in seconds: three tile rows."""
    p = workloads.rff_problem(3000, 384, 10, seed=3, q=64)
    got = gu.cv(p, "interp", want_W=False)
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
    _check_cv(got, want)
    gote = gu.cv(p, "exact", want_W=False)
    wante = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid)
    _check_cv(gote, wante)


@pytest.mark.parametrize("d,form", [(1536, 0), (1537, 0), (1700, 0), (1800, 0),
                                    (1800, 1)])
def test_cv_interp_around_overlap_threshold(gu, d, form):
    """Above twelve tile columns the fit and the diagonal-block inverses of
    the finished columns, and the forward solve steps that need only them,
    run on a second stream while the last twelve columns are factored: at
    d=1536 (twelve columns) nothing is forked, at 1537 one column is (the
    thirteenth is a one-row ragged tile; no forward step can start early),
    at 1700 two (one early forward step), at 1800 three (two).  With the
    stacked solve form (form 1) only the fit and the inverses are forked."""
    B = gu.B
    p = workloads.gaussian_problem(2 * d + 7, d, 3, seed=21, g=4, q=8)
    B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, form)
    try:
        got = gu.cv(p, "interp")
    finally:
        B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, 0)
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True)
    _check_cv(got, want)


def test_cv_interp_is_exact_when_samples_are_the_grid(gu):
    p = workloads.gaussian_problem(600, 40, 3, seed=5, q=4, lam_range=(1e-2, 1.0))
    gi = gu.cv(p, "interp", lam_s=p.lam_grid, r=3)
    ge = gu.cv(p, "exact")
    np.testing.assert_allclose(gi["mse"], ge["mse"], rtol=1e-9)


def test_cv_flags_nonpositive_interpolated_pivot(gu):
    """Far outside the samples a high-degree fit can drive a diagonal entry
    of the interpolated factor negative: both sides flag the same (fold,
    lambda) units."""
    p = workloads.gaussian_problem(400, 30, 2, seed=4, g=4, q=6)
    lam_s = np.array([1.0, 2.0, 3.0, 4.0]) * p.scale
    # a cubic through sqrt-like curves sampled on [1, 4] turns negative when
    # extrapolated to -2
    lam_grid = np.array([-2.0, 0.5, 1.5, 2.5, 3.5, 5.0]) * p.scale
    got = gu.cv(p, "interp", lam_s=lam_s, lam_grid=lam_grid, r=3)
    want = oracle.cv_interp(p.X, p.Y, p.k, lam_s, lam_grid, 3, want_W=True)
    assert np.any(want["flags"] & 2)
    np.testing.assert_array_equal(got["flags"] & 2, want["flags"] & 2)
    ok = want["flags"] == 0
    np.testing.assert_allclose(got["mse"][ok], want["mse"][ok], rtol=1e-8)


def test_cv_is_deterministic(gu):
    p = workloads.gaussian_problem(900, 200, 10, seed=8, g=4, q=16)
    a = gu.cv(p, "interp")
    b = gu.cv(p, "interp")
    np.testing.assert_array_equal(a["mse"], b["mse"])
    np.testing.assert_array_equal(a["W"], b["W"])


def test_argument_errors(gu):
    B = gu.B
    p = B.make_problem(100, 10, 2, 5, g=3, r=3, q=4)  # r >= g
    with pytest.raises(B.PicholError) as e:
        B.pichol_workspace_size(p, B.PICHOL_METHOD_INTERP)
    assert e.value.status == B.PICHOL_ERR_ARG
    p = B.make_problem(100, 10, 2, 5, g=3, r=2, q=4)
    nbytes = B.pichol_workspace_size(p, B.PICHOL_METHOD_INTERP)
    w = gu.ws(16)
    err = gu.empty(20)
    info = gu.empty(15, torch.int32)
    flags = gu.empty(20, torch.int32)
    with pytest.raises(B.PicholError) as e:
        B.pichol_cv_interp(p, [0.1, 0.2, 0.3], [0.1] * 4, 0.3, w, 16, err, None, info, flags)
    assert e.value.status == B.PICHOL_ERR_WORKSPACE
    w = gu.ws(nbytes)
    with pytest.raises(B.PicholError) as e:  # repeated sample value
        B.pichol_cv_interp(p, [0.1, 0.1, 0.3], [0.1] * 4, 0.3, w, nbytes, err, None, info,
                           flags)
    assert e.value.status == B.PICHOL_ERR_ARG


@pytest.mark.parametrize("method", ["interp", "exact"])
@pytest.mark.parametrize("group", [2, 3, 4])
def test_cv_with_lookahead_matches_without(gu, method, group):
    """The side-stream look-ahead schedule gives bitwise the same results
    (same kernels, same per-tile accumulation order).  The order is chosen
    so that several groups run their trailing updates on the side stream
    (ceil(d/128) = 2 * group + 2 tiles)."""
    B = gu.B
    d = 128 * (2 * group + 2) - 50
    p = workloads.rff_problem(2 * d + 600, d, 10, seed=6, g=5, q=12)
    old_group = B.pichol_get_option(B.PICHOL_OPT_PANEL_GROUP)
    B.pichol_set_option(B.PICHOL_OPT_PANEL_GROUP, group)
    B.pichol_set_option(B.PICHOL_OPT_LOOKAHEAD, 0)
    try:
        a = gu.cv(p, method)
        B.pichol_set_option(B.PICHOL_OPT_LOOKAHEAD, 1)
        b = gu.cv(p, method)
    finally:
        B.pichol_set_option(B.PICHOL_OPT_LOOKAHEAD, 0)
        B.pichol_set_option(B.PICHOL_OPT_PANEL_GROUP, old_group)
    np.testing.assert_array_equal(a["mse"], b["mse"])
    np.testing.assert_array_equal(a["W"], b["W"])
    if group == 2:
        want = (oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
                if method == "interp" else oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid))
        np.testing.assert_allclose(b["mse"], want["mse"], rtol=1e-10)
