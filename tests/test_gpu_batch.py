"""Batched cross-validation of many independent problems (pichol_cv_batch)
against the oracle and against the single-problem pipeline, through the
C-ABI.

Inputs: problems of uneven d (several tiles, ragged tails), c in {1, 3},
different n (so different fold sizes and scales) inside one bucket, and
buckets of one problem.  Hold-out errors match the oracle at the FP64 bar
(1e-10 relative); a problem's results match its own single-problem run to
1e-13 (the bucket shares its first problem's scaled lambda values, which
may differ from another problem's in the last few bits) and exactly where
those values coincide.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gu(gpu):
    import gpu_util
    return gpu_util


def small_batch():
    mk = workloads.gaussian_problem
    return [
        mk(700, 130, 3, seed=11, g=4, r=2, q=9),
        mk(650, 130, 3, seed=12, g=4, r=2, q=9),   # same bucket, other n
        mk(900, 256, 1, seed=13, g=4, r=2, q=9),
        mk(400, 100, 3, seed=14, g=4, r=2, q=9),
        mk(800, 130, 1, seed=15, g=4, r=2, q=9),   # same d, other c
        mk(720, 130, 3, seed=16, g=4, r=2, q=9),   # third member of bucket 0
    ]


@pytest.fixture(scope="module")
def interp_run(gu):
    probs = small_batch()
    run = gu.BatchRun(probs, "interp")
    return probs, run, run.run()


def test_batch_forms_the_expected_buckets(gu, interp_run):
    probs, run, _ = interp_run
    assert gu.B.pichol_batch_buckets(run.batch, run.method) == 4


def test_batch_interp_matches_oracle(gu, interp_run):
    probs, run, got = interp_run
    for i, (p, o) in enumerate(zip(probs, got)):
        want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r, want_W=True)
        assert np.all(o["info"] == 0) and np.all(o["flags"] == 0), i
        np.testing.assert_allclose(o["mse"], want["mse"], rtol=1e-10, atol=0,
                                   err_msg=f"problem {i}")
        scale = np.abs(want["W"]).max()
        assert np.abs(o["W"] - want["W"]).max() <= 1e-9 * scale, i


def test_batch_interp_matches_single_pipeline(gu, interp_run):
    probs, run, got = interp_run
    for i, (p, o) in enumerate(zip(probs, got)):
        one = gu.cv(p, "interp")
        np.testing.assert_allclose(o["mse"], one["mse"], rtol=1e-13, atol=0)
        np.testing.assert_array_equal(o["info"], one["info"])
        np.testing.assert_array_equal(o["flags"], one["flags"])
    # the first problem of each bucket supplies the shared scaled values, so
    # its results are the single-problem results bit for bit
    for i in [0, 2, 3, 4]:
        np.testing.assert_array_equal(got[i]["mse"], gu.cv(probs[i], "interp")["mse"])


def test_batch_exact_matches_oracle_and_single(gu):
    probs = small_batch()[:4]
    run = gu.BatchRun(probs, "exact")
    got = run.run()
    for i, (p, o) in enumerate(zip(probs, got)):
        want = oracle.cv_exact(p.X, p.Y, p.k, p.lam_grid)
        assert np.all(o["info"] == 0) and np.all(o["flags"] == 0)
        np.testing.assert_allclose(o["mse"], want["mse"], rtol=1e-10, atol=0)
        one = gu.cv(p, "exact")
        np.testing.assert_array_equal(o["mse"], one["mse"])
        np.testing.assert_array_equal(o["W"], one["W"])


@pytest.mark.parametrize("tune", [dict(streams=1, order=0), dict(streams=2, order=1),
                                  dict(streams=4, order=0)])
def test_batch_schedule_does_not_change_results(gu, interp_run, tune):
    probs, run, ref = interp_run
    run.clear()
    got = run.run(tune)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a["mse"], b["mse"])
        np.testing.assert_array_equal(a["W"], b["W"])
        np.testing.assert_array_equal(a["flags"], b["flags"])


@pytest.mark.parametrize("form", [1, 2])
def test_batch_solve_form_per_bucket(gu, interp_run, form):
    """A solve form chosen per d bucket through the tuning record: results
    within rounding of the default run, and against the oracle."""
    probs, run, ref = interp_run
    run.clear()
    nts = sorted({(p.d + 127) // 128 for p in probs})
    got = run.run(dict(streams=2, order=0, solve_form={nt: form for nt in nts}))
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a["mse"], b["mse"], rtol=1e-12, atol=0)
        np.testing.assert_array_equal(a["flags"], b["flags"])
    p = probs[0]
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
    np.testing.assert_allclose(got[0]["mse"], want["mse"], rtol=1e-10, atol=0)


def test_batch_mixed_precision_equals_single_mixed(gu):
    probs = small_batch()[2:4]
    run = gu.BatchRun(probs, "interp", precision=gu.B.PICHOL_PREC_MIXED)
    got = run.run()
    for p, o in zip(probs, got):
        one = gu.cv(p, "interp", precision=gu.B.PICHOL_PREC_MIXED)
        np.testing.assert_array_equal(o["mse"], one["mse"])


def test_batch_graph_replays_match_eager(gu, interp_run):
    probs, run, ref = interp_run
    g = gu.B.pichol_cv_batch_graph(run.batch, run.method, None, run.ws, run.nbytes)
    try:
        for rep in range(3):
            run.clear()
            # eager work of the program's own between the replays
            junk = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
            float(junk.sum())
            gu.B.pichol_graph_launch(g)
            torch.cuda.synchronize()
            got = run.results()
            for a, b in zip(got, ref):
                np.testing.assert_array_equal(a["mse"], b["mse"], err_msg=f"replay {rep}")
                np.testing.assert_array_equal(a["W"], b["W"])
                np.testing.assert_array_equal(a["info"], b["info"])
                np.testing.assert_array_equal(a["flags"], b["flags"])
    finally:
        gu.B.pichol_graph_destroy(g)


def test_batch_rejects_bad_items(gu):
    probs = small_batch()[:2]
    run = gu.BatchRun(probs, "interp")
    run.batch.items[1].p.refine = 1
    with pytest.raises(gu.B.PicholError):
        gu.B.pichol_cv_batch(run.batch, run.method, None, run.ws, run.nbytes)
    run.batch.items[1].p.refine = 0
    with pytest.raises(gu.B.PicholError) as e:
        gu.B.pichol_cv_batch(run.batch, run.method, None, run.ws, run.nbytes - 1)
    assert e.value.status == gu.B.PICHOL_ERR_WORKSPACE
    with pytest.raises(gu.B.PicholError):
        gu.B.pichol_cv_batch(run.batch, run.method, dict(streams=5), run.ws, run.nbytes)


@pytest.mark.parametrize("n,d", [(900, 300), (3700, 1800)])
def test_captured_single_problem_stage_replays_match_eager(gu, n, d):
    """pichol_graph_begin/end around the piCholesky stage of one problem:
    replays equal the eager call bit for bit, with eager work between.  At
    d = 1800 (15 tile columns) the eager call forks its second stream and
    the captured one does not."""
    B = gu.B
    p = workloads.gaussian_problem(n, d, 3, seed=31, g=5, r=2, q=11)
    prob = B.make_problem(p.n, p.d, p.c, p.k, p.g, p.r, p.q, True)
    nb = B.pichol_workspace_size(prob, B.PICHOL_METHOD_INTERP)
    w = gu.ws(nb)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        err = gu.empty(p.k * p.q)
        W = gu.empty(p.k * p.q * p.d * p.c)
        info = gu.empty(p.k * p.g, torch.int32)
        flags = gu.empty(p.k * p.q, torch.int32)
        B.pichol_cv_gram(prob, gu.dev(p.X), gu.dev(p.Y), w, nb)
        B.pichol_cv_interp(prob, p.lam_s, p.lam_grid, p.lam_ref, w, nb, err, W, info, flags)
        s.synchronize()
        ref = (err.cpu().numpy(), W.cpu().numpy(), flags.cpu().numpy())
        B.pichol_graph_begin()
        B.pichol_cv_interp(prob, p.lam_s, p.lam_grid, p.lam_ref, w, nb, err, W, info, flags)
        g = B.pichol_graph_end()
    try:
        for rep in range(3):
            err.fill_(float("nan"))
            W.fill_(float("nan"))
            torch.cuda.synchronize()
            junk = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
            float(junk.sum())
            B.pichol_graph_launch(g, s)
            s.synchronize()
            np.testing.assert_array_equal(err.cpu().numpy(), ref[0], err_msg=f"replay {rep}")
            np.testing.assert_array_equal(W.cpu().numpy(), ref[1])
            np.testing.assert_array_equal(flags.cpu().numpy(), ref[2])
    finally:
        B.pichol_graph_destroy(g)
    want = oracle.cv_interp(p.X, p.Y, p.k, p.lam_s, p.lam_grid, p.r)
    np.testing.assert_allclose(ref[0].reshape(p.k, p.q), want["mse"], rtol=1e-10, atol=0)
