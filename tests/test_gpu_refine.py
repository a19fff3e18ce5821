"""Iterative refinement of the solves (pichol_problem.refine) against the
oracle's orc_refine, through the pipeline calls.

FP64: the refined hold-out errors and weights of both methods match the
oracle run with the same number of steps at the FP64 bar (1e-10 relative
on hold-out errors), on inputs with several tiles and a ragged tail.

Mixed precision: refinement against H_f + lambda I is the classic remedy
for a lower-precision factor.  Each step contracts the error by about
kappa * |E| / |A| (about 1e-4 here), so two steps bring the exact method's
results back to the FP64 oracle's at the same 1e-10 bar.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


@pytest.fixture(scope="module")
def prob():
    return workloads.gaussian_problem(1500, 520, 5, seed=3, g=5, r=2, q=12)


def _wclose(got, want, rel):
    scale = np.abs(want).max()
    diff = np.abs(got - want).max()
    assert diff <= rel * scale, f"max diff {diff:.3e} > {rel:.0e} * {scale:.3e}"


@pytest.mark.parametrize("steps", [1, 3])
def test_refined_interp_matches_oracle(gu, prob, steps):
    got = gu.cv(prob, "interp", refine=steps)
    want = oracle.cv_interp(prob.X, prob.Y, prob.k, prob.lam_s, prob.lam_grid, prob.r,
                            want_W=True, refine=steps)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=1e-10, atol=0)
    _wclose(got["W"], want["W"], 1e-9)
    # refinement moved the result: it differs from the unrefined one
    base = oracle.cv_interp(prob.X, prob.Y, prob.k, prob.lam_s, prob.lam_grid, prob.r)
    assert np.max(np.abs(got["mse"] - base["mse"]) / base["mse"]) > 1e-9


def test_refined_exact_matches_oracle(gu, prob):
    got = gu.cv(prob, "exact", refine=1)
    want = oracle.cv_exact(prob.X, prob.Y, prob.k, prob.lam_grid, want_W=True, refine=1)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=1e-10, atol=0)
    _wclose(got["W"], want["W"], 1e-9)


def test_mixed_exact_refined_reaches_fp64(gu, prob):
    want = oracle.cv_exact(prob.X, prob.Y, prob.k, prob.lam_grid, want_W=True)
    raw = gu.cv(prob, "exact", precision=gu.B.PICHOL_PREC_MIXED)
    ref = gu.cv(prob, "exact", precision=gu.B.PICHOL_PREC_MIXED, refine=2)
    assert np.all(ref["info"] == 0) and np.all(ref["flags"] == 0)
    e_raw = np.max(np.abs(raw["mse"] - want["mse"]) / want["mse"])
    e_ref = np.max(np.abs(ref["mse"] - want["mse"]) / want["mse"])
    print(f"mixed exact: rel err {e_raw:.2e} unrefined, {e_ref:.2e} after 2 steps")
    np.testing.assert_allclose(ref["mse"], want["mse"], rtol=1e-10, atol=0)
    _wclose(ref["W"], want["W"], 1e-9)


def test_refined_interp_converges_toward_exact(gu, prob):
    ex = oracle.cv_exact(prob.X, prob.Y, prob.k, prob.lam_grid)
    gaps = []
    for steps in [0, 2, 6]:
        got = gu.cv(prob, "interp", refine=steps, want_W=False)
        gaps.append(np.max(np.abs(got["mse"] - ex["mse"]) / ex["mse"]))
    print("interp vs exact after 0/2/6 steps:", ["%.2e" % g for g in gaps])
    assert gaps[1] < gaps[0] and gaps[2] < gaps[1]


def test_refined_interp_past_overlap_threshold(gu):
    """Refinement after a call that forked its second stream (d = 1700:
    the fit, inverses and early forward steps of the first columns ran
    beside the last columns' factorization, and the correction solves
    follow the join)."""
    p = workloads.gaussian_problem(3407, 1700, 3, seed=21, g=4, r=2, q=8)
    got = gu.cv(p, "interp", refine=1)
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True,
                            refine=1)
    assert np.all(got["info"] == 0) and np.all(got["flags"] == 0)
    np.testing.assert_allclose(got["mse"], want["mse"], rtol=1e-10, atol=0)
    _wclose(got["W"], want["W"], 1e-9)
