"""Seeded synthetic inputs for piCholesky cross-validation.

This module only draws inputs: design matrices, label columns and the lambda
grids.  It holds none of the method's arithmetic and serves the oracle, the
tests and the benchmark alike, so both sides of every comparison receive the
very same arrays.

The paper's experiments project MNIST, COIL-100 and Caltech-101/256 through
random feature maps (Sec. 6.1); those datasets are not available here, so the
workloads below stand in for them with data of the same structure: Gaussian
designs with decaying column scales, and random Fourier features of uniform
inputs.  Every array is drawn from ``numpy.random.default_rng(seed)``
(PCG64) in FP64, in the order the recipe lists.

Lambda grids: ``s = trace(X^T X / n) / d`` over the full X, and
``lam = s * 10**linspace(log10(lo), log10(hi), m)`` with both ends included,
for the sample values (m = g) and the dense grid (m = q).  The paper draws
its candidates as exponentially spaced values over a per-dataset range
(Sec. 6.3) and does not say which of them are sampled; the samples here are
log-spaced over the same range.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    X: np.ndarray          # n x d, float64, C-contiguous
    Y: np.ndarray          # n x c, float64 (+1 / -1)
    k: int                 # folds
    g: int                 # sample lambdas
    r: int                 # polynomial degree
    lam_s: np.ndarray      # g sample lambdas (ascending)
    lam_grid: np.ndarray   # q grid lambdas (ascending)
    scale: float           # s = trace(X^T X / n) / d
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def d(self) -> int:
        return self.X.shape[1]

    @property
    def c(self) -> int:
        return self.Y.shape[1]

    @property
    def q(self) -> int:
        return self.lam_grid.shape[0]

    @property
    def lam_ref(self) -> float:
        return float(np.max(self.lam_s))


def lam_scale(X: np.ndarray) -> float:
    """s = trace(X^T X / n) / d, i.e. the mean squared entry of X."""
    n, d = X.shape
    return float(np.einsum("ij,ij->", X, X) / (n * d))


def log_grid(scale: float, lo: float, hi: float, m: int) -> np.ndarray:
    return scale * 10.0 ** np.linspace(np.log10(lo), np.log10(hi), m)


def one_vs_all(cls: np.ndarray, c: int) -> np.ndarray:
    Y = -np.ones((cls.shape[0], c))
    Y[np.arange(cls.shape[0]), cls] = 1.0
    return Y


def gaussian_problem(n: int, d: int, c: int = 10, seed: int = 0, k: int = 5,
                     g: int = 4, r: int = 2, q: int = 31,
                     lam_range=(1e-4, 1e1), name: str | None = None) -> Problem:
    """Gaussian design: X ~ N(0,1)^{n x d}, column j scaled by
    1/sqrt(1 + j/16); teacher W0 ~ N(0,1)^{d x c}; class = argmax(X W0);
    labels +1 for the class, -1 otherwise (c = 1: sign of X w0)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    X *= 1.0 / np.sqrt(1.0 + np.arange(d) / 16.0)
    W0 = rng.standard_normal((d, c))
    if c == 1:
        Y = np.where(X @ W0 >= 0.0, 1.0, -1.0)
    else:
        Y = one_vs_all(np.argmax(X @ W0, axis=1), c)
    s = lam_scale(X)
    return Problem(name or f"gauss_n{n}_d{d}_c{c}", np.ascontiguousarray(X),
                   np.ascontiguousarray(Y), k, g, r,
                   log_grid(s, *lam_range, g), log_grid(s, *lam_range, q), s,
                   {"kind": "gaussian", "seed": seed, "lam_range": lam_range})


def lowres_problem(n: int = 3000, d: int = 384, c: int = 10, seed: int = 7,
                   k: int = 5, g: int = 6, r: int = 2, q: int = 31,
                   noise: float = 1e-3, lam_range=(1e-6, 1e1),
                   name: str | None = None) -> Problem:
    """A well-fitted regression target (the hold-out residual far below the
    labels): X ~ N(0,1)^{n x d} with column j scaled by 1/sqrt(1 + j/16);
    teacher W0 ~ N(0,1)^{d x c}, each column rescaled so that the column of
    X W0 has unit standard deviation; Y = X W0 + noise * N(0,1)^{n x c}.
    At the small lambdas of the range, |Y_v - X_v W|^2 / |Y_v|^2 is about
    noise^2.  Draw order: X, W0, the noise."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    X *= 1.0 / np.sqrt(1.0 + np.arange(d) / 16.0)
    W0 = rng.standard_normal((d, c))
    W0 /= (X @ W0).std(axis=0)
    Y = X @ W0 + noise * rng.standard_normal((n, c))
    s = lam_scale(X)
    return Problem(name or f"lowres_n{n}_d{d}_c{c}", np.ascontiguousarray(X),
                   np.ascontiguousarray(Y), k, g, r,
                   log_grid(s, *lam_range, g), log_grid(s, *lam_range, q), s,
                   {"kind": "lowres", "seed": seed, "noise": noise,
                    "lam_range": lam_range})


def rff_problem(n: int, d: int, c: int = 10, seed: int = 0, k: int = 5,
                g: int = 6, r: int = 2, q: int = 64, p: int = 784,
                sigma: float = 5.0, lam_range=(1e-6, 1e0),
                name: str | None = None, chunk: int = 8192) -> Problem:
    """Random Fourier features of uniform inputs: Z ~ U[0,1]^{n x p},
    W ~ N(0, 1/sigma^2)^{p x d}, b ~ U[0, 2 pi]^d,
    X = sqrt(2/d) cos(Z W + b); teacher T0 ~ N(0,1)^{p x c},
    class = argmax((Z - 1/2) T0); labels +1 / -1 one-vs-all."""
    rng = np.random.default_rng(seed)
    Z = rng.random((n, p))
    W = rng.standard_normal((p, d)) / sigma
    b = rng.random(d) * (2.0 * np.pi)
    T0 = rng.standard_normal((p, c))
    X = np.empty((n, d))
    amp = np.sqrt(2.0 / d)
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        blk = Z[r0:r1] @ W
        blk += b
        np.cos(blk, out=blk)
        blk *= amp
        X[r0:r1] = blk
    cls = np.argmax((Z - 0.5) @ T0, axis=1)
    Y = one_vs_all(cls, c)
    s = lam_scale(X)
    return Problem(name or f"rff_n{n}_d{d}_c{c}", X, Y, k, g, r,
                   log_grid(s, *lam_range, g), log_grid(s, *lam_range, q), s,
                   {"kind": "rff", "seed": seed, "p": p, "sigma": sigma,
                    "lam_range": lam_range})


def powerlaw_problem(d: int, c: int, seed: int, k: int = 5, g: int = 5,
                     r: int = 2, q: int = 32, lam_range=(1e-4, 1e1),
                     name: str | None = None) -> Problem:
    """One problem of the many-problem workload: n = 8 d rows,
    X ~ N(0,1)^{n x d} with column j (1-based) scaled by j^{-1/2};
    teacher W0 ~ N(0,1)^{d x c}; c = 10: one-vs-all labels of
    argmax(X W0); c = 1: sign(X w0).  Draw order: X, then W0."""
    return _powerlaw(np.random.default_rng(seed), d, c, seed, k, g, r, q,
                     lam_range, name)


def _powerlaw(rng, d, c, seed, k, g, r, q, lam_range, name):
    n = 8 * d
    X = rng.standard_normal((n, d))
    X *= 1.0 / np.sqrt(np.arange(1, d + 1, dtype=np.float64))
    W0 = rng.standard_normal((d, c))
    if c == 1:
        Y = np.where(X @ W0 >= 0.0, 1.0, -1.0)
    else:
        Y = one_vs_all(np.argmax(X @ W0, axis=1), c)
    s = lam_scale(X)
    return Problem(name or f"plaw_d{d}_c{c}_s{seed}", np.ascontiguousarray(X),
                   np.ascontiguousarray(Y), k, g, r,
                   log_grid(s, *lam_range, g), log_grid(s, *lam_range, q), s,
                   {"kind": "powerlaw", "seed": seed, "lam_range": lam_range})


BATCH_DS = (256, 384, 512, 768, 1024, 1536, 2048)


def batch_problems(count: int = 48, seed0: int = 1000, ds=BATCH_DS,
                   cs=(1, 10), **kw) -> list[Problem]:
    """The many-problem workload: problem p uses one generator seeded
    seed0 + p, which draws d uniformly from ds, then c uniformly from cs,
    then the problem's arrays as in powerlaw_problem (X, then W0)."""
    opts = dict(k=5, g=5, r=2, q=32, lam_range=(1e-4, 1e1))
    opts.update(kw)
    out = []
    for p in range(count):
        rng = np.random.default_rng(seed0 + p)
        d = int(rng.choice(ds))
        c = int(rng.choice(cs))
        out.append(_powerlaw(rng, d, c, seed0 + p, opts["k"], opts["g"],
                             opts["r"], opts["q"], opts["lam_range"],
                             f"plaw{p}_d{d}_c{c}"))
    return out


WORKLOADS = ("gauss_n2000_d256", "rff_n20000_d2048", "rff_n60000_d4096")


def named(name: str) -> Problem:
    """The named workloads of the parity tests and the benchmark.

    gauss_n2000_d256: Gaussian, n=2000, d=256, c=10, k=5, g=4, r=2, q=31,
        range [1e-4, 1e1]
    rff_n20000_d2048: random Fourier features, n=20000, d=2048, c=10, k=5,
        g=6, r=2, q=64, range [1e-6, 1]
    rff_n60000_d4096: random Fourier features, n=60000, d=4096, c=10, k=5,
        g=6, r=2, q=64, range [1e-6, 1] (the benchmark workload)
    """
    if name == "gauss_n2000_d256":
        return gaussian_problem(2000, 256, 10, seed=0, g=4, r=2, q=31,
                                lam_range=(1e-4, 1e1), name=name)
    if name == "rff_n20000_d2048":
        return rff_problem(20000, 2048, 10, seed=0, g=6, r=2, q=64, name=name)
    if name == "rff_n60000_d4096":
        return rff_problem(60000, 4096, 10, seed=0, g=6, r=2, q=64, name=name)
    raise ValueError(f"unknown workload {name!r}; known: {', '.join(WORKLOADS)}")
