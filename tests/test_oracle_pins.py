"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself: a
closed form, a library routine (LAPACK through numpy/scipy), the SVD form of
ridge regression the paper states in Sec. 6.2, polynomial reproduction and
interpolation properties of the least-squares fit of Algorithm 1, or an
invariant of the whole pipeline.  The cases are chosen so that a dropped term,
a wrong sign or index, or a transposed operand fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
import workloads

EPS = np.finfo(np.float64).eps


def spd(d, seed, cond=100.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    ev = np.logspace(0, -np.log10(cond), d)
    return (Q * ev) @ Q.T


# ------------------------------------------------------------------ folds / Gram

@pytest.mark.parametrize("n,k", [(10, 5), (11, 5), (2048, 5), (7, 3), (2, 2)])
def test_fold_bounds_match_array_split(n, k):
    sizes = [len(a) for a in np.array_split(np.arange(n), k)]
    b = oracle.fold_bounds(n, k)
    assert list(np.diff(b)) == sizes
    assert b[0] == 0 and b[-1] == n


@pytest.mark.parametrize("normalize", [True, False])
def test_fold_gram_bruteforce(normalize):
    rng = np.random.default_rng(1)
    n, d, c, k = 53, 7, 3, 5
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((n, c))
    b = oracle.fold_bounds(n, k)
    Gsum = np.zeros((d, d))
    for f in range(k):
        H, B, ntr = oracle.fold_gram(X, Y, k, f, normalize)
        mask = np.ones(n, bool)
        mask[b[f]:b[f + 1]] = False
        Xt, Yt = X[mask], Y[mask]
        s = 1.0 / ntr if normalize else 1.0
        assert ntr == mask.sum()
        np.testing.assert_allclose(H, Xt.T @ Xt * s, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(B, Xt.T @ Yt * s, rtol=1e-13, atol=1e-14)
        assert np.array_equal(H, H.T)
        Xv = X[b[f]:b[f + 1]]
        Gsum += Xv.T @ Xv
    # the validation blocks tile the rows: their Grams add up to the full one
    np.testing.assert_allclose(Gsum, X.T @ X, rtol=1e-12)


# ------------------------------------------------------------------ Cholesky

def test_cholesky_1x1():
    L, info = oracle.cholesky(np.array([[3.0]]), 1.5)
    assert info == 0
    assert L[0, 0] == np.sqrt(4.5)


@pytest.mark.parametrize("a,b,c,lam", [(4.0, 2.0, 3.0, 1.0), (2.0, -1.5, 5.0, 0.25),
                                       (1e-3, 1e-4, 2e-3, 1e-6)])
def test_cholesky_2x2_closed_form(a, b, c, lam):
    A = np.array([[a, b], [b, c]])
    L, info = oracle.cholesky(A, lam)
    assert info == 0
    l11 = np.sqrt(a + lam)
    l21 = b / l11
    l22 = np.sqrt(c + lam - b * b / (a + lam))
    np.testing.assert_allclose(L, [[l11, 0.0], [l21, l22]], rtol=4 * EPS)


def test_cholesky_diagonal_closed_form():
    h = np.array([0.5, 2.0, 1e-3, 7.0, 0.0])
    L, info = oracle.cholesky(np.diag(h), 0.3)
    assert info == 0
    np.testing.assert_allclose(L, np.diag(np.sqrt(h + 0.3)), rtol=2 * EPS)


@pytest.mark.parametrize("d,seed,lam", [(1, 0, 0.1), (9, 1, 1e-3), (37, 2, 0.0),
                                        (64, 3, 1e-5), (130, 4, 2.0)])
def test_cholesky_matches_lapack(d, seed, lam):
    A = spd(d, seed, cond=1e3)
    L, info = oracle.cholesky(A, lam)
    assert info == 0
    Lref = np.linalg.cholesky(A + lam * np.eye(d))
    np.testing.assert_allclose(L, Lref, rtol=0, atol=1e-12 * np.abs(Lref).max())
    assert np.all(np.triu(L, 1) == 0.0)
    assert np.all(np.diag(L) > 0)


@pytest.mark.parametrize("d", [5, 40, 200])
def test_cholesky_backward_error(d):
    A = spd(d, 10 + d, cond=1e6)
    lam = 1e-7
    L, info = oracle.cholesky(A, lam)
    assert info == 0
    Al = A + lam * np.eye(d)
    resid = np.linalg.norm(L @ L.T - Al, 2)
    assert resid <= 4 * d * EPS * np.linalg.norm(Al, 2)


def test_cholesky_reads_lower_triangle_only():
    A = spd(6, 5)
    junk = A.copy()
    junk[np.triu_indices(6, 1)] = 1e6
    L1, _ = oracle.cholesky(A, 0.1)
    L2, _ = oracle.cholesky(junk, 0.1)
    assert np.array_equal(L1, L2)


def test_cholesky_not_positive_definite_reports_first_column():
    # leading minors of order 1, 2 are positive, order 3 is not
    A = np.diag([1.0, 2.0, -1.0, 4.0])
    assert oracle.cholesky(A, 0.5)[1] == 3
    assert oracle.cholesky(A, 1.5)[1] == 0
    B = np.array([[1.0, 2.0], [2.0, 1.0]])  # indefinite: 1 - 4 < 0
    assert oracle.cholesky(B, 0.0)[1] == 2
    assert oracle.cholesky(np.array([[np.nan]]), 0.0)[1] == 1


def test_pack_roundtrip():
    rng = np.random.default_rng(3)
    L = np.tril(rng.standard_normal((9, 9)))
    t = oracle.pack_lower(L)
    assert t.shape == (45,)
    assert t[3 * 4 // 2 + 2] == L[3, 2]
    assert np.array_equal(oracle.unpack_lower(t, 9), L)


# ------------------------------------------------------------------ fit / evaluate

def _quadratic_targets(lam, D, seed, deg=2):
    """Target rows whose every entry is a polynomial of degree deg in lambda."""
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal((deg + 1, D))
    V = np.vander(lam, deg + 1, increasing=True)
    return V @ coef, coef


@pytest.mark.parametrize("g,r", [(3, 2), (4, 2), (6, 2), (5, 3), (4, 1), (3, 0)])
def test_fit_reproduces_polynomials(g, r):
    lam_s = np.array([0.05, 0.3, 0.9, 1.7, 2.2, 3.1])[:g]
    T, coef = _quadratic_targets(lam_s, 11, seed=g, deg=r)
    lam_ref = 2.5
    Theta = oracle.fit(T, lam_s, r, lam_ref)
    for lam in [0.0, 0.07, 1.0, 2.9, 4.0]:
        want = np.vander([lam], r + 1, increasing=True)[0] @ coef
        np.testing.assert_allclose(oracle.evaluate(Theta, lam, lam_ref), want,
                                   rtol=1e-11, atol=1e-11)
    # coefficients are in tau = lambda / lam_ref
    np.testing.assert_allclose(Theta, coef * (lam_ref ** np.arange(r + 1))[:, None],
                               rtol=1e-10, atol=1e-11)


@pytest.mark.parametrize("g", [2, 3, 4, 6])
def test_fit_interpolates_samples_when_degree_is_g_minus_1(g):
    rng = np.random.default_rng(20 + g)
    lam_s = np.sort(rng.uniform(0.01, 1.0, g))
    T = rng.standard_normal((g, 17))
    Theta = oracle.fit(T, lam_s, g - 1, lam_s.max())
    # Algorithm 1 solves the normal equations, whose rounding error grows
    # with cond(V)^2
    cond = np.linalg.cond(np.vander(lam_s / lam_s.max(), g, increasing=True))
    tol = 10 * cond ** 2 * EPS * np.abs(T).max()
    for s in range(g):
        np.testing.assert_allclose(oracle.evaluate(Theta, lam_s[s], lam_s.max()),
                                   T[s], rtol=0, atol=tol)


def test_fit_is_the_least_squares_solution():
    rng = np.random.default_rng(7)
    g, r, D = 6, 2, 23
    lam_s = np.logspace(-3, 0, g)
    T = rng.standard_normal((g, D))
    lam_ref = lam_s.max()
    Theta = oracle.fit(T, lam_s, r, lam_ref)
    V = np.vander(lam_s / lam_ref, r + 1, increasing=True)
    # normal-equation residual V^T (T - V Theta) = 0
    np.testing.assert_allclose(V.T @ (T - V @ Theta), 0.0, atol=1e-12)
    # LAPACK least squares (QR/SVD based) gives the same polynomial
    ref, *_ = np.linalg.lstsq(V, T, rcond=None)
    np.testing.assert_allclose(Theta, ref, rtol=1e-10, atol=1e-12)


def test_fit_does_not_depend_on_basis_scale():
    rng = np.random.default_rng(8)
    lam_s = np.array([1e-3, 1e-2, 0.1, 1.0])
    T = rng.standard_normal((4, 13))
    a = oracle.fit(T, lam_s, 2, 1.0)
    b = oracle.fit(T, lam_s, 2, 0.37)
    for lam in [5e-4, 0.05, 0.6]:
        np.testing.assert_allclose(oracle.evaluate(a, lam, 1.0),
                                   oracle.evaluate(b, lam, 0.37), rtol=1e-11,
                                   atol=1e-12)


def test_fit_rejects_bad_arguments():
    T = np.ones((3, 4))
    with pytest.raises(ValueError):
        oracle.fit(T, [0.1, 0.2, 0.3], 3, 1.0)  # r >= g
    with pytest.raises(ValueError):
        oracle.fit(T, [0.1, 0.1, 0.3], 2, 1.0)  # repeated sample
    with pytest.raises(ValueError):
        oracle.fit(T, [0.1, 0.2, 0.3], 1, 0.0)  # lam_ref <= 0


def test_interpolated_factor_tracks_exact_factor():
    """Sec. 3.3 / Fig. 2: second-order polynomials through a few exact factors
    trace the factor entries closely between the samples."""
    A = spd(8, 30, cond=50.0)
    lam_s = np.array([0.1, 0.2, 0.35, 0.5, 0.7])
    T = np.stack([oracle.pack_lower(oracle.cholesky(A, l)[0]) for l in lam_s])
    Theta = oracle.fit(T, lam_s, 2, 0.7)
    spread = np.linalg.norm(T[-1] - T[0])
    for lam in [0.15, 0.3, 0.6]:
        exact = oracle.pack_lower(oracle.cholesky(A, lam)[0])
        approx = oracle.evaluate(Theta, lam, 0.7)
        err = np.linalg.norm(approx - exact)
        assert err <= 1e-2 * np.linalg.norm(exact)
        assert err <= 0.05 * spread


@pytest.mark.parametrize("g", [4, 6])
def test_interpolation_error_is_cubic_in_the_sample_width(g):
    """Sec. 4 main result: with the g samples within w of lambda_c and the
    evaluation point within gamma <= w of it, the RMS error of the degree-2
    piCholesky factor is bounded by a multiple of w^3 (gamma^3 and
    w^3 (1 + gamma^2) terms, R and |V^+| bounded as w shrinks).  Halving w
    (and gamma = w/2 with it) must divide the error by about 8; a fit of too
    low a degree, a dropped coefficient or a wrong sample abscissa would
    divide it by 4 or less."""
    A = spd(4, 41, cond=20.0)
    lam_c = 0.5
    D = 4 * 5 // 2
    errs = []
    for w in [0.16, 0.08, 0.04, 0.02]:
        lam_s = lam_c + w * np.linspace(-1.0, 1.0, g)
        T = np.stack([oracle.pack_lower(oracle.cholesky(A, l)[0]) for l in lam_s])
        Theta = oracle.fit(T, lam_s, 2, lam_s.max())
        lam = lam_c + 0.5 * w
        exact = oracle.pack_lower(oracle.cholesky(A, lam)[0])
        errs.append(np.linalg.norm(oracle.evaluate(Theta, lam, lam_s.max())
                                   - exact) / np.sqrt(D))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 6.5) and np.all(ratios < 9.5), ratios
    # the degree-1 fit of the same samples only reaches second order
    w = 0.02
    lam_s = lam_c + w * np.linspace(-1.0, 1.0, g)
    T = np.stack([oracle.pack_lower(oracle.cholesky(A, l)[0]) for l in lam_s])
    lin = oracle.fit(T, lam_s, 1, lam_s.max())
    exact = oracle.pack_lower(oracle.cholesky(A, lam_c + 0.5 * w)[0])
    e1 = np.linalg.norm(oracle.evaluate(lin, lam_c + 0.5 * w, lam_s.max())
                        - exact) / np.sqrt(D)
    assert e1 > 20 * errs[-1]


# ------------------------------------------------------------------ solves / hold-out

def test_solve_diagonal_closed_form():
    Ld = np.diag([2.0, 0.5, 3.0])
    B = np.array([[1.0, 2.0], [3.0, -1.0], [0.5, 0.25]])
    W, fl = oracle.solve(Ld, B)
    assert fl == 0
    np.testing.assert_allclose(W, B / np.diag(Ld)[:, None] ** 2, rtol=2 * EPS)


@pytest.mark.parametrize("d,c", [(1, 1), (12, 3), (70, 10)])
def test_solve_matches_lapack_triangular(d, c):
    rng = np.random.default_rng(d)
    L = np.linalg.cholesky(spd(d, d + 100, cond=1e3))
    B = rng.standard_normal((d, c))
    W, fl = oracle.solve(L, B)
    assert fl == 0
    U = scipy.linalg.solve_triangular(L, B, lower=True)
    Wref = scipy.linalg.solve_triangular(L.T, U, lower=False)
    np.testing.assert_allclose(W, Wref, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(L @ (L.T @ W), B, atol=1e-10)


def test_solve_flags():
    L = np.array([[1.0, 0.0], [0.5, -2.0]])
    _, fl = oracle.solve(L, np.ones(2))
    assert fl & 2
    L0 = np.array([[1.0, 0.0], [0.5, 0.0]])
    _, fl = oracle.solve(L0, np.ones(2))
    assert fl == 3  # zero pivot: not positive and a non-finite solution


def test_holdout_definition_and_gram_identity():
    rng = np.random.default_rng(4)
    nv, d, c = 31, 6, 3
    Xv = rng.standard_normal((nv, d))
    Yv = np.sign(rng.standard_normal((nv, c)))
    W = rng.standard_normal((d, c))
    R = Yv - Xv @ W
    sse = oracle.holdout_sse(Xv, Yv, W)
    np.testing.assert_allclose(sse, np.sum(R * R), rtol=1e-13)
    # sum R^2 = |Y|^2 - 2 <W, X^T Y> + tr(W^T X^T X W)
    ident = np.sum(Yv * Yv) - 2 * np.sum(W * (Xv.T @ Yv)) + np.sum(W * (Xv.T @ Xv @ W))
    np.testing.assert_allclose(sse, ident, rtol=1e-12)
    sst = oracle.holdout_sst(Yv)
    np.testing.assert_allclose(sst, np.sum((Yv - Yv.mean(0)) ** 2), rtol=1e-13)


def test_factor_nrmse_pins():
    """NRMSE section: predicting every entry of the factor by its mean gives
    exactly 1; an exact fit gives 0; the numerator is linear in the error
    and entries above the diagonal are ignored."""
    rng = np.random.default_rng(21)
    d = 9
    L = np.tril(rng.standard_normal((d, d)))
    E = np.tril(rng.standard_normal((d, d)))
    il = np.tril_indices(d)
    assert oracle.factor_nrmse(L, L) == 0.0
    mean = np.full((d, d), L[il].mean())
    np.testing.assert_allclose(oracle.factor_nrmse(np.tril(mean), L), 1.0, rtol=1e-14)
    base = oracle.factor_nrmse(L + E, L)
    for delta in (0.5, -3.0, 1e-6):
        np.testing.assert_allclose(oracle.factor_nrmse(L + delta * E, L),
                                   abs(delta) * base, rtol=1e-9)
    # a common affine map of the entries leaves the ratio unchanged
    np.testing.assert_allclose(oracle.factor_nrmse(np.tril(2.5 * (L + E) - 7.0),
                                                   np.tril(2.5 * L - 7.0)), base, rtol=1e-12)
    junk = np.triu(rng.standard_normal((d, d)), 1)
    assert oracle.factor_nrmse(L + E + junk, L - junk) == base


def test_cv_nrmse_pins():
    """Hold-out NRMSE: predicting each validation label by its fold's column
    mean gives 1, an exact prediction gives 0."""
    rng = np.random.default_rng(22)
    n, d, c, k = 53, 4, 3, 5
    X = rng.standard_normal((n, d))
    X[:, 0] = 1.0
    Y = np.sign(rng.standard_normal((n, c)))
    b = oracle.fold_bounds(n, k)
    sse = np.zeros((k, 2))
    for f in range(k):
        Xv, Yv = X[b[f]:b[f + 1]], Y[b[f]:b[f + 1]]
        W = np.zeros((d, c))
        W[0] = Yv.mean(0)              # the column means, through the ones column
        sse[f, 0] = oracle.holdout_sse(Xv, Yv, W)
        Wx = rng.standard_normal((d, c))
        sse[f, 1] = oracle.holdout_sse(Xv, Xv @ Wx, Wx)   # labels fitted exactly
    nr = oracle.cv_nrmse(Y, k, sse)
    np.testing.assert_allclose(nr[:, 0], 1.0, rtol=1e-13)
    np.testing.assert_allclose(nr[:, 1], 0.0, atol=1e-13)


# ------------------------------------------------------------------ pipelines

def _ridge_svd(Xt, Yt, lam, ntr):
    """Sec. 6.2 closed form theta = V diag(sig/(sig^2+lam)) U^T y, applied to
    the normalised training data X_tr/sqrt(n_tr), Y_tr/sqrt(n_tr)."""
    Xs = Xt / np.sqrt(ntr)
    Ys = Yt / np.sqrt(ntr)
    U, sig, Vt = np.linalg.svd(Xs, full_matrices=False)
    return Vt.T @ ((sig / (sig ** 2 + lam))[:, None] * (U.T @ Ys))


@pytest.mark.parametrize("n,d,c,k", [(60, 5, 2, 3), (203, 17, 4, 5), (41, 40, 1, 2)])
def test_exact_cv_matches_svd_ridge_form(n, d, c, k):
    p = workloads.gaussian_problem(n, d, c, seed=n, k=k, q=7)
    out = oracle.cv_exact(p.X, p.Y, k, p.lam_grid, want_W=True)
    b = oracle.fold_bounds(n, k)
    assert np.all(out["info"] == 0) and np.all(out["flags"] == 0)
    for f in range(k):
        mask = np.ones(n, bool)
        mask[b[f]:b[f + 1]] = False
        Xt, Yt = p.X[mask], p.Y[mask]
        Xv, Yv = p.X[~mask], p.Y[~mask]
        for t, lam in enumerate(p.lam_grid):
            th = _ridge_svd(Xt, Yt, lam, mask.sum())
            scale = np.abs(th).max()
            np.testing.assert_allclose(out["W"][f, t], th, rtol=0,
                                       atol=1e-9 * scale)
            mse = np.sum((Yv - Xv @ th) ** 2) / (Yv.size)
            np.testing.assert_allclose(out["mse"][f, t], mse, rtol=1e-9)


def test_fold_exact_matches_svd_ridge_form_and_cv_exact():
    """The one-fold exact path (from numpy-formed H_f, B_f) against the SVD
    ridge form and the whole-CV oracle on the same fold; a non-PD shift gives
    the same info, NaN and flag pattern as cv_exact."""
    n, d, c, k = 203, 17, 4, 5
    p = workloads.gaussian_problem(n, d, c, seed=n, k=k, q=7)
    b = oracle.fold_bounds(n, k)
    lam = np.concatenate([p.lam_grid, [-1e3]])
    full = oracle.cv_exact(p.X, p.Y, k, lam, want_W=True)
    for f in [0, 3]:
        mask = np.ones(n, bool)
        mask[b[f]:b[f + 1]] = False
        Xt, Yt, Xv, Yv = p.X[mask], p.Y[mask], p.X[~mask], p.Y[~mask]
        H, Bm = Xt.T @ Xt / mask.sum(), Xt.T @ Yt / mask.sum()
        out = oracle.fold_exact(H, Bm, Xv, Yv, lam, want_W=True)
        np.testing.assert_array_equal(out["info"], full["info"][f])
        np.testing.assert_array_equal(out["flags"], full["flags"][f])
        assert out["info"][-1] == 1 and np.isnan(out["mse"][-1])
        assert np.all(np.isnan(out["W"][-1]))
        np.testing.assert_allclose(out["mse"][:-1], full["mse"][f, :-1], rtol=1e-12)
        for t, l in enumerate(p.lam_grid):
            th = _ridge_svd(Xt, Yt, l, mask.sum())
            np.testing.assert_allclose(out["W"][t], th, rtol=0,
                                       atol=1e-9 * np.abs(th).max())
            mse = np.sum((Yv - Xv @ th) ** 2) / Yv.size
            np.testing.assert_allclose(out["mse"][t], mse, rtol=1e-9)


def test_interp_equals_exact_when_samples_are_the_grid():
    """With g = q, the samples equal to the grid and r = g - 1 the fit
    interpolates every exact factor, so piCholesky CV is exact CV."""
    p = workloads.gaussian_problem(300, 24, 3, seed=5, q=4, lam_range=(1e-2, 1.0))
    ex = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid, want_W=True)
    pi = oracle.cv_interp(p.X, p.Y, p.k, p.lam_grid, p.lam_grid, 3, want_W=True)
    np.testing.assert_allclose(pi["mse"], ex["mse"], rtol=1e-9)
    np.testing.assert_allclose(pi["W"], ex["W"], rtol=0, atol=1e-8 * np.abs(ex["W"]).max())


@pytest.mark.parametrize("g,r", [(4, 3), (6, 2)])
def test_interp_cv_off_sample_matches_library_composition(g, r):
    """piCholesky CV (sec. 4: exact factors at the samples, an entry-wise
    polynomial of degree r in lambda fitted by least squares, evaluated off
    the samples, then the two triangular solves and the hold-out error) at
    grid values between and beyond the samples, against the same steps done
    with independent library routines: LAPACK Cholesky of the normalised
    training Gram, numpy's polyfit/polyval on every entry, LAPACK triangular
    solves and the residual of the validation rows."""
    from numpy.polynomial import polynomial as P
    p = workloads.gaussian_problem(180, 12, 3, seed=31, k=3, g=g, q=9,
                                   lam_range=(1e-2, 2.0))
    lam_s = np.geomspace(0.03, 1.5, g)
    lam_grid = np.concatenate([np.geomspace(0.012, 1.9, 8), [2.5]])
    out = oracle.cv_interp(p.X, p.Y, p.k, lam_s, lam_grid, r, want_W=True)
    b = oracle.fold_bounds(p.n, p.k)
    x = lam_s / lam_s.max()
    for f in range(p.k):
        mask = np.ones(p.n, bool)
        mask[b[f]:b[f + 1]] = False
        Xt, Yt, Xv, Yv = p.X[mask], p.Y[mask], p.X[~mask], p.Y[~mask]
        ntr = mask.sum()
        H, B = Xt.T @ Xt / ntr, Xt.T @ Yt / ntr
        Ls = np.stack([np.linalg.cholesky(H + lam * np.eye(p.d)) for lam in lam_s])
        coef = P.polyfit(x, Ls.reshape(g, -1), r)  # (r+1) x d^2
        for t, lam in enumerate(lam_grid):
            L = P.polyval(lam / lam_s.max(), coef).reshape(p.d, p.d)
            L = np.tril(L)
            z = scipy.linalg.solve_triangular(L, B, lower=True)
            w = scipy.linalg.solve_triangular(L.T, z, lower=False)
            np.testing.assert_allclose(out["W"][f, t], w, rtol=0,
                                       atol=1e-9 * np.abs(w).max())
            mse = np.sum((Yv - Xv @ w) ** 2) / Yv.size
            np.testing.assert_allclose(out["mse"][f, t], mse, rtol=1e-9)


def test_interp_cv_reproduces_sample_points():
    """At grid values that coincide with samples, r = g - 1 reproduces the
    exact hold-out errors even when the rest of the grid is interpolated."""
    p = workloads.gaussian_problem(400, 30, 2, seed=9, g=4, q=10, lam_range=(1e-3, 1.0))
    lam_s = p.lam_grid[[0, 3, 6, 9]]
    ex = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid)
    pi = oracle.cv_interp(p.X, p.Y, p.k, lam_s, p.lam_grid, 3)
    np.testing.assert_allclose(pi["mse"][:, [0, 3, 6, 9]], ex["mse"][:, [0, 3, 6, 9]],
                               rtol=1e-9)


def test_fold_interp_matches_cv_interp():
    p = workloads.gaussian_problem(250, 20, 3, seed=2, g=4, q=9)
    full = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True)
    b = oracle.fold_bounds(p.n, p.k)
    for f in [0, 4]:
        H, B, _ = oracle.fold_gram(p.X, p.Y, p.k, f)
        one = oracle.fold_interp(H, B, p.X[b[f]:b[f + 1]], p.Y[b[f]:b[f + 1]],
                                 p.lam_s, p.lam_grid, p.r, want_W=True)
        np.testing.assert_array_equal(one["mse"], full["mse"][f])
        np.testing.assert_array_equal(one["W"], full["W"][f])


def test_not_pd_sample_sets_info_and_nan():
    rng = np.random.default_rng(0)
    n, d = 40, 6
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((n, 1))
    # a negative sample lambda larger than the smallest eigenvalue of H_f
    lam_s = np.array([-50.0, 0.1, 0.2])
    out = oracle.cv_interp(X, Y, 2, lam_s, np.array([0.15]), 2, lam_ref=0.2)
    assert np.all(out["info"][:, 0] > 0)
    assert np.all(np.isnan(out["mse"]))
    assert np.all(out["flags"] & 1)


def test_selection_helpers():
    curve = np.array([3.0, 1.0, 1.0, np.nan, 2.0])
    assert oracle.select(curve) == 1  # ties go to the smallest lambda
    g = oracle.gaps(np.array([1.0, 0.5, 2.0]), np.array([1.0, 0.6, 0.4]),
                    np.array([0.1, 1.0, 10.0]))
    assert g["t_pi"] == 1 and g["t_ex"] == 2
    np.testing.assert_allclose(g["regret"], 0.2)
    np.testing.assert_allclose(g["sel_err_log10"], 1.0)
    np.testing.assert_allclose(g["curve_gap"], 4.0)
    # smallest interpolated minus smallest exact, relative to the latter
    np.testing.assert_allclose(g["min_gap"], (0.5 - 0.4) / 0.4)


def test_gauss_n2000_d256_matches_known_behaviour():
    """Gaussian workload n=2000, d=256: piCholesky selects the same grid
    value as exact CV and its curve stays within 1% of it."""
    p = workloads.named("gauss_n2000_d256")
    ex = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid)
    pi = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
    g = oracle.gaps(oracle.cv_curve(pi["mse"]), oracle.cv_curve(ex["mse"]), p.lam_grid)
    assert g["t_pi"] == g["t_ex"]
    assert g["curve_gap"] < 1e-2
    # at the sample values (grid indices 0, 10, 20, 30) the fit of degree 2
    # through 4 samples is not an interpolant, but stays close
    np.testing.assert_allclose(p.lam_s, p.lam_grid[[0, 10, 20, 30]], rtol=1e-12)


def test_cholesky_derivative_matches_frechet_form():
    """Thm. 4.1: the derivative of the factor along Delta = I is the
    lower-triangular Gamma with Gamma L^T + L Gamma^T = I, i.e.
    Gamma = L Phi(L^-1 L^-T) where Phi keeps the strict lower triangle and half
    the diagonal.  Central differences of the oracle's factor must agree."""
    A = spd(7, 40, cond=20.0)
    lam, h = 0.3, 1e-5
    L, _ = oracle.cholesky(A, lam)
    fd = (oracle.cholesky(A, lam + h)[0] - oracle.cholesky(A, lam - h)[0]) / (2 * h)
    Li = np.linalg.inv(L)
    S = Li @ Li.T
    Phi = np.tril(S, -1) + 0.5 * np.diag(np.diag(S))
    Gamma = L @ Phi
    np.testing.assert_allclose(Gamma @ L.T + L @ Gamma.T, np.eye(7), atol=1e-12)
    np.testing.assert_allclose(fd, Gamma, rtol=0, atol=1e-8)


# ------------------------------------------------------------------ iterative refinement

def _perturbed_factor(H, lam, rel, seed):
    L, info = oracle.cholesky(H, lam)
    assert info == 0
    rng = np.random.default_rng(seed)
    return np.tril(L * (1.0 + rel * rng.standard_normal(L.shape)))


@pytest.mark.parametrize("lam", [1e-3, 0.3])
def test_refine_converges_to_lapack_solution(lam):
    """Residual correction with an approximate factor converges
    geometrically to the LAPACK solution of (H + lam I) W = B; a wrong
    sign of the shift or a transposed product would stall it."""
    d, c = 45, 3
    H = spd(d, 7, cond=50.0)
    rng = np.random.default_rng(8)
    B = rng.standard_normal((d, c))
    Lp = _perturbed_factor(H, lam, 1e-2, 9)
    W0, fl = oracle.solve(Lp, B)
    assert fl == 0
    want = scipy.linalg.solve(H + lam * np.eye(d), B, assume_a="pos")
    errs = []
    for m in [0, 1, 2, 3, 12]:
        W, fl = oracle.refine(H, lam, Lp, B, W0, m)
        assert fl == 0
        errs.append(np.max(np.abs(W - want)) / np.max(np.abs(want)))
    assert errs[0] > 1e-3
    for a, b in zip(errs[:3], errs[1:4]):
        assert b < 0.3 * a
    assert errs[-1] < 1e-12


def test_refine_with_exact_factor_only_moves_by_rounding():
    d, c, lam = 30, 2, 0.1
    H = spd(d, 3)
    B = np.random.default_rng(4).standard_normal((d, c))
    L, _ = oracle.cholesky(H, lam)
    W0, _ = oracle.solve(L, B)
    W1, fl = oracle.refine(H, lam, L, B, W0, 3)
    assert fl == 0
    assert np.max(np.abs(W1 - W0)) <= 100 * EPS * np.max(np.abs(W0)) * 50.0
    W2, _ = oracle.refine(H, lam, L, B, W0, 0)
    np.testing.assert_array_equal(W2, W0)


def test_refined_interp_cv_converges_to_exact_cv():
    """Refinement against H_f + lambda_t I pulls the interpolated solutions
    to the exact ones: after enough steps piCholesky CV equals exact CV."""
    p = workloads.gaussian_problem(300, 24, 3, seed=6, g=4, q=9)
    ex = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid, want_W=True)
    pi0 = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True)
    pi2 = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True,
                           refine=2)
    # the worst grid value of this problem contracts by about 0.27 per step
    pi30 = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True,
                            refine=30)
    scale = np.abs(ex["W"]).max()
    e0 = np.abs(pi0["W"] - ex["W"]).max() / scale
    e2 = np.abs(pi2["W"] - ex["W"]).max() / scale
    e30 = np.abs(pi30["W"] - ex["W"]).max() / scale
    assert e0 > 1e-3 and e2 < 0.1 * e0 and e30 < 1e-12
    np.testing.assert_allclose(pi30["mse"], ex["mse"], rtol=1e-11)
    # exact factors: refinement changes the hold-out errors only by rounding
    ex2 = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid, refine=2)
    np.testing.assert_allclose(ex2["mse"], ex["mse"], rtol=1e-12)


def test_refined_fold_interp_matches_cv_interp():
    p = workloads.gaussian_problem(250, 20, 3, seed=2, g=4, q=9)
    full = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True,
                            refine=2)
    b = oracle.fold_bounds(p.n, p.k)
    H, B, _ = oracle.fold_gram(p.X, p.Y, p.k, 1)
    one = oracle.fold_interp(H, B, p.X[b[1]:b[2]], p.Y[b[1]:b[2]], p.lam_s,
                             p.lam_grid, p.r, want_W=True, refine=2)
    np.testing.assert_array_equal(one["mse"], full["mse"][1])


# ------------------------------------------------------------------ gradient of the hold-out error

def test_eval_deriv_is_the_polynomial_derivative():
    rng = np.random.default_rng(3)
    Theta = rng.standard_normal((3, 11))
    lam_ref, lam, h = 2.0, 0.7, 1e-5
    num = (oracle.evaluate(Theta, lam + h, lam_ref)
           - oracle.evaluate(Theta, lam - h, lam_ref)) / (2 * h)
    # a quadratic: the central difference is exact up to rounding
    np.testing.assert_allclose(oracle.evaluate_deriv(Theta, lam, lam_ref), num,
                               rtol=1e-8, atol=1e-9)
    tau = lam / lam_ref
    want = (Theta[1] + 2 * tau * Theta[2]) / lam_ref
    np.testing.assert_allclose(oracle.evaluate_deriv(Theta, lam, lam_ref), want,
                               rtol=1e-14, atol=1e-15)


def _fd_dlog(fn, lam_grid, h=1e-4):
    return (fn(lam_grid * np.exp(h)) - fn(lam_grid * np.exp(-h))) / (2 * h)


def test_interp_gradient_matches_central_differences():
    p = workloads.gaussian_problem(300, 24, 3, seed=6, g=4, q=9)
    got = oracle.cv_grad(p.X, p.Y, p.k, p.lam_grid, p.lam_s, p.r)
    assert np.all(got["flags"] == 0)
    fd = _fd_dlog(lambda lg: oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, lg, p.r,
                                              lam_ref=p.lam_ref)["mse"], p.lam_grid)
    scale = np.abs(got["dlog"]).max()
    assert np.abs(fd - got["dlog"]).max() <= 1e-6 * scale
    ref = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
    np.testing.assert_array_equal(got["mse"], ref["mse"])


def test_exact_gradient_matches_svd_closed_form():
    """d mse / d lambda from the SVD form of ridge regression:
    theta = V diag(s/(s^2+lam)) U^T y, d theta/d lam = -V diag(s/(s^2+lam)^2) U^T y."""
    n, d, c, k = 203, 17, 4, 5
    p = workloads.gaussian_problem(n, d, c, seed=21, k=k, q=7)
    got = oracle.cv_grad(p.X, p.Y, k, p.lam_grid)
    b = oracle.fold_bounds(n, k)
    for f in range(k):
        mask = np.ones(n, bool)
        mask[b[f]:b[f + 1]] = False
        Xt, Yt = p.X[mask] / np.sqrt(mask.sum()), p.Y[mask] / np.sqrt(mask.sum())
        Xv, Yv = p.X[~mask], p.Y[~mask]
        U, sig, Vt = np.linalg.svd(Xt, full_matrices=False)
        UtY = U.T @ Yt
        for t, lam in enumerate(p.lam_grid):
            th = Vt.T @ ((sig / (sig ** 2 + lam))[:, None] * UtY)
            dth = -Vt.T @ ((sig / (sig ** 2 + lam) ** 2)[:, None] * UtY)
            R = Yv - Xv @ th
            dmse = -2.0 * np.sum(R * (Xv @ dth)) / Yv.size
            np.testing.assert_allclose(got["dlog"][f, t], lam * dmse, rtol=1e-8,
                                       atol=1e-12)
    fd = _fd_dlog(lambda lg: oracle.cv_exact(p.X, p.Y, k, lg)["mse"], p.lam_grid)
    assert np.abs(fd - got["dlog"]).max() <= 1e-6 * np.abs(got["dlog"]).max()


def test_gradient_scale_error_would_be_caught():
    """The central-difference check is sharp: a gradient off by a factor of
    two (as from a dropped symmetric term of dA = dL L^T + L dL^T when the
    two terms are close) misses it by far more than its tolerance."""
    p = workloads.gaussian_problem(300, 24, 3, seed=6, g=4, q=9)
    got = oracle.cv_grad(p.X, p.Y, p.k, p.lam_grid, p.lam_s, p.r)
    fd = _fd_dlog(lambda lg: oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, lg, p.r,
                                              lam_ref=p.lam_ref)["mse"], p.lam_grid)
    assert np.abs(fd - 0.5 * got["dlog"]).max() > 1e-2 * np.abs(fd).max()


# ------------------------------------------------------------------ the paper's variants (PINRMSE, MChol)

def test_pinrmse_matches_numpy_polyfit():
    """PINRMSE replaces T by the g-vector of sample hold-out errors: per
    fold, the least-squares polynomial in tau through those errors, which
    numpy's polyfit computes independently."""
    from numpy.polynomial import polynomial as P
    p = workloads.gaussian_problem(300, 24, 3, seed=6, g=4, q=9)
    pr = oracle.pinrmse(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
    ex = oracle.cv_exact(p.X, p.Y, p.k, p.lam_s)
    np.testing.assert_allclose(pr["mse_samples"], ex["mse"], rtol=1e-14)
    tau_s, tau_t = p.lam_s / p.lam_ref, p.lam_grid / p.lam_ref
    for f in range(p.k):
        co = P.polyfit(tau_s, pr["mse_samples"][f], p.r)
        np.testing.assert_allclose(pr["mse"][f], P.polyval(tau_t, co), rtol=1e-11)


def test_pinrmse_interpolates_when_degree_is_g_minus_1():
    p = workloads.gaussian_problem(250, 20, 2, seed=7, g=4, q=10, lam_range=(1e-3, 1.0))
    lam_s = p.lam_grid[[0, 3, 6, 9]]
    pr = oracle.pinrmse(p.X, p.Y, p.k, lam_s, p.lam_grid, 3)
    ex = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid)
    np.testing.assert_allclose(pr["mse"][:, [0, 3, 6, 9]], ex["mse"][:, [0, 3, 6, 9]],
                               rtol=1e-9)


def test_mchol_bracketing_search():
    """MChol halves s from 1.5 until s <= 0.0025 (10 levels), recentres on
    the best of three points at every level, and ends next to the minimiser
    of a dense exact search over the initial range."""
    p = workloads.gaussian_problem(300, 24, 3, seed=6, g=4, q=9)
    c0 = np.log10(p.scale) - 1.5
    m = oracle.mchol(p.X, p.Y, p.k, c0, 1.5, 0.0025)
    assert len(m["trace"]) == 10
    s = 1.5
    for lvl, (lams, cvv) in enumerate(m["trace"]):
        np.testing.assert_allclose(np.log10(lams[2]) - np.log10(lams[1]), s, rtol=1e-12)
        if lvl > 0:
            prev_l, prev_v = m["trace"][lvl - 1]
            np.testing.assert_allclose(lams[1], prev_l[np.argmin(prev_v)], rtol=1e-12)
        s /= 2
    dense = np.logspace(c0 - 1.5, c0 + 1.5, 601)
    cv = oracle.cv_exact(p.X, p.Y, p.k, dense)["mse"].mean(0)
    assert abs(m["log10_lam"] - np.log10(dense[np.argmin(cv)])) <= 0.01


# ------------------------------------------------------------------ vectorisation orders (Sec. 5)

def test_recursive_order_small_case_from_the_text():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "recursive_order_h4_h0_2.txt")
    want = [tuple(int(v) for v in ln.split()) for ln in open(path)
            if ln.strip() and not ln.startswith("#")]
    assert oracle.recursive_order(4, 2) == want


@pytest.mark.parametrize("h,h0", [(16, 4), (37, 5), (64, 64), (9, 1)])
def test_recursive_order_is_a_bijection_on_the_triangle(h, h0):
    order = oracle.recursive_order(h, h0)
    assert len(order) == h * (h + 1) // 2
    assert set(order) == {(i, j) for i in range(h) for j in range(i + 1)}
    if h <= h0:  # no split: the row-wise order of pack_lower
        assert order == [(i, j) for i in range(h) for j in range(i + 1)]


# ------------------------------------------------------------------ log-lambda basis (optional variant)

def test_log_basis_fit_matches_polyfit_and_reproduces_polynomials():
    from numpy.polynomial import polynomial as P
    rng = np.random.default_rng(11)
    g, r, D = 6, 2, 9
    lam_s = np.logspace(-6, 0, g) * 3e-4
    lam_ref = lam_s.max()
    u = np.log(lam_s / lam_ref)
    T = rng.standard_normal((g, D))
    th = oracle.fit(T, lam_s, r, lam_ref, basis=1)
    for e in range(D):
        np.testing.assert_allclose(th[:, e], P.polyfit(u, T[:, e], r), rtol=1e-9, atol=1e-12)
    # targets that are quadratics in log(lambda) are reproduced anywhere
    coef = rng.standard_normal((3, D))
    Tq = np.stack([coef[0] + coef[1] * x + coef[2] * x * x for x in u])
    thq = oracle.fit(Tq, lam_s, r, lam_ref, basis=1)
    lam = 7.3e-7
    x = np.log(lam / lam_ref)
    np.testing.assert_allclose(oracle.evaluate(thq, lam, lam_ref, basis=1),
                               coef[0] + coef[1] * x + coef[2] * x * x, rtol=1e-9)


def test_log_basis_derivative_matches_central_differences():
    rng = np.random.default_rng(12)
    Theta = rng.standard_normal((3, 7))
    lam_ref, lam, h = 2.0, 0.03, 1e-7
    num = (oracle.evaluate(Theta, lam + h, lam_ref, basis=1)
           - oracle.evaluate(Theta, lam - h, lam_ref, basis=1)) / (2 * h)
    np.testing.assert_allclose(oracle.evaluate_deriv(Theta, lam, lam_ref, basis=1), num,
                               rtol=1e-6)


def test_log_basis_cv_interpolates_samples_and_gradient_matches_differences():
    p = workloads.gaussian_problem(400, 30, 2, seed=9, g=4, q=10, lam_range=(1e-3, 1.0))
    lam_s = p.lam_grid[[0, 3, 6, 9]]
    pi = oracle.cv_interp(p.X, p.Y, p.k, lam_s, p.lam_grid, 3, basis=1)
    ex = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid)
    np.testing.assert_allclose(pi["mse"][:, [0, 3, 6, 9]], ex["mse"][:, [0, 3, 6, 9]],
                               rtol=1e-8)
    q = workloads.gaussian_problem(300, 24, 3, seed=6, g=4, q=9)
    got = oracle.cv_grad(q.X, q.Y, q.k, q.lam_grid, q.lam_s, q.r, basis=1)
    fd = _fd_dlog(lambda lg: oracle.cv_interp(q.X, q.Y, q.k, q.lam_s, lg, q.r,
                                              lam_ref=q.lam_ref, basis=1)["mse"], q.lam_grid)
    assert np.abs(fd - got["dlog"]).max() <= 1e-6 * np.abs(got["dlog"]).max()


def test_parity_bar_is_attainable_on_the_parity_workloads():
    """Two backward-stable FP64 solvers of H_f + lambda I agree to about
    kappa * eps * (a low power of d).  On the workloads the GPU parity tests
    hold to 1e-10 (Gaussian n=2000, d=256; random features n=3000, d=384),
    kappa * eps * d stays below 1e-11 for every fold at the smallest grid
    value, so the bar leaves room for rounding-order differences.  The fit's
    basis in tau = lambda/lam_ref is well conditioned where raw lambda is
    not (the random-feature scale puts lambda near 1e-10 .. 1e-4)."""
    eps = np.finfo(np.float64).eps
    for p in (workloads.gaussian_problem(2000, 256, 10, seed=0, g=4, r=2, q=31),
              workloads.rff_problem(3000, 384, 10, seed=3, q=64)):
        n, d = p.X.shape
        starts = np.cumsum([0] + [len(a) for a in np.array_split(np.arange(n), p.k)])
        lam0 = float(p.lam_grid.min())
        for f in range(p.k):
            keep = np.ones(n, bool)
            keep[starts[f]:starts[f + 1]] = False
            Xt = p.X[keep]
            ev = np.linalg.eigvalsh(Xt.T @ Xt / Xt.shape[0])
            kappa = (ev[-1] + lam0) / (ev[0] + lam0)
            assert kappa * eps * d < 1e-11, (p.name, f, kappa)
        V = np.vander(p.lam_s / p.lam_ref, p.r + 1, increasing=True)
        assert np.linalg.cond(V) < 1e3
    V_raw = np.vander(p.lam_s, p.r + 1, increasing=True)
    assert np.linalg.cond(V_raw) > 1e6


def test_interpolated_cv_matches_50_digit_arithmetic():
    """The oracle's whole piCholesky CV (fold Gram matrices, sample
    factorizations, the least-squares fit in tau, evaluation at grid values
    between and beyond the samples, the two substitutions and the hold-out
    MSE) against the same mathematics carried out in 50-digit arithmetic
    (mpmath) at d = 6.  The interpolated factor is linear in the sample
    factors, Lhat(tau) = sum_s w_s(tau) L_s with w(tau) = phi(tau)^T V^+, and
    the solution is (Lhat Lhat^T)^{-1} B_f; kappa(H_f + lambda I) is about
    10 here, so FP64 agrees to well inside 1e-10."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(11)
    n, d, c, k, g, r = 40, 6, 2, 4, 4, 2
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((n, c))
    lam_s = np.array([0.05, 0.1, 0.2, 0.4])
    lam_grid = np.array([0.03, 0.07, 0.15, 0.3, 0.6])
    got = oracle.cv_interp(X, Y, k, lam_s, lam_grid, r, want_W=True)
    starts = np.cumsum([0] + [len(a) for a in np.array_split(np.arange(n), k)])
    lam_ref = mp.mpf(float(lam_s.max()))
    tau_s = [mp.mpf(float(x)) / lam_ref for x in lam_s]
    V = mp.matrix([[t ** j for j in range(r + 1)] for t in tau_s])
    Vp = (V.T * V) ** -1 * V.T  # the pseudo-inverse, (r+1) x g
    Xm = [[mp.mpf(float(x)) for x in row] for row in X]
    Ym = [[mp.mpf(float(y)) for y in row] for row in Y]
    for f in range(k):
        val = range(starts[f], starts[f + 1])
        keep = [i for i in range(n) if i not in val]
        H = mp.matrix(d, d)
        B = mp.matrix(d, c)
        for i in keep:
            for a in range(d):
                for b in range(d):
                    H[a, b] += Xm[i][a] * Xm[i][b]
                for j in range(c):
                    B[a, j] += Xm[i][a] * Ym[i][j]
        H /= len(keep)
        B /= len(keep)
        Ls = [mp.cholesky(H + mp.mpf(float(lam)) * mp.eye(d)) for lam in lam_s]
        for t, lam in enumerate(lam_grid):
            tau = mp.mpf(float(lam)) / lam_ref
            w = [sum(Vp[j, s] * tau ** j for j in range(r + 1)) for s in range(g)]
            Lh = mp.matrix(d, d)
            for a in range(d):
                for b in range(a + 1):
                    Lh[a, b] = sum(w[s] * Ls[s][a, b] for s in range(g))
            A = Lh * Lh.T
            sse = mp.mpf(0)
            for j in range(c):
                wj = mp.lu_solve(A, B[:, j])
                np.testing.assert_allclose(
                    got["W"][f, t, :, j], [float(x) for x in wj], rtol=1e-10,
                    atol=1e-10 * float(mp.norm(wj, mp.inf)))
                for i in val:
                    res = Ym[i][j] - sum(Xm[i][a] * wj[a] for a in range(d))
                    sse += res * res
            want = float(sse / (len(val) * c))
            assert abs(got["mse"][f, t] - want) <= 1e-10 * want, (f, t)


@pytest.mark.parametrize("w", [0.2, 0.05])
def test_interpolation_error_within_main_result_bound(w):
    """The Sec. 4 main result at a tiny size (A of order 4): with g samples
    in [lam_c - w, lam_c + w] and lam_c > gamma >= w, the degree-2 factor
    from the oracle's fit and evaluation satisfies, for lambda in
    [lam_c - gamma, lam_c + gamma],
        ||C(A + lambda I) - p(lambda)||_F
            <= [gamma^3 + sqrt(g) w^3 (1 + gamma^2)(lam_c + 1) ||V^+||_2] R,
    with V the raw-lambda Vandermonde matrix of the samples and
    R = max_s (||M^-1 E||^2 ||M^-1 v_I|| + ||M^-1|| ||M^-1 E|| ||M^-1 v_I||^2)
    over [lam_c - gamma, lam_c + gamma], M = L_s (x) I + I (x) L_s,
    E = K (x) I + I (x) K, K = vec^-1(M^-1 v_I), all taken literally from the
    paper (the maximum over s by a grid of 81 points).  The bound is loose
    (the error reaches about 1% of it, where the fit extrapolates furthest
    from samples within w = 0.05)."""
    rng = np.random.default_rng(5)
    n = 4
    Bm = rng.standard_normal((n, n + 2))
    A = Bm @ Bm.T / (n + 2) + 0.1 * np.eye(n)
    lam_c, gam, g, r = 1.0, 0.4, 5, 2
    lam_s = np.linspace(lam_c - w, lam_c + w, g)
    lam_ref = float(lam_s.max())
    T = np.stack([oracle.pack_lower(oracle.cholesky(A, float(x))[0]) for x in lam_s])
    Th = oracle.fit(T, lam_s, r, lam_ref)
    I = np.eye(n)
    vI = I.reshape(-1, order="F")

    def r_term(s):
        L = np.linalg.cholesky(A + s * I)
        Mi = np.linalg.inv(np.kron(L, I) + np.kron(I, L))
        x = Mi @ vI
        K = x.reshape(n, n, order="F")
        ME = Mi @ (np.kron(K, I) + np.kron(I, K))
        nx = np.linalg.norm(x)
        return (np.linalg.norm(ME, 2) ** 2 * nx
                + np.linalg.norm(Mi, 2) * np.linalg.norm(ME, 2) * nx ** 2)

    R = max(r_term(s) for s in np.linspace(lam_c - gam, lam_c + gam, 81))
    Vp = np.linalg.norm(np.linalg.pinv(np.vander(lam_s, r + 1, increasing=True)), 2)
    bound = (gam ** 3 + np.sqrt(g) * w ** 3 * (1 + gam ** 2) * (lam_c + 1) * Vp) * R
    for lam in np.linspace(lam_c - gam, lam_c + gam, 9):
        p = oracle.unpack_lower(oracle.evaluate(Th, float(lam), lam_ref), n)
        err = np.linalg.norm(np.linalg.cholesky(A + lam * I) - p)
        assert err <= bound, (lam, err, bound)
