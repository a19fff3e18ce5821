"""The C-ABI library loads on a machine without a GPU and exports every
function include/pichol.h declares; host-only entry points (sizes, layout
arithmetic, argument validation) behave as documented.  No compute call is
made here."""
import ctypes
import os
import re

import pytest

from paper_1404_0466_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pichol.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pichol_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libpichol.so is not built (python -m paper_1404_0466_amd.build)")
    return B.load()


def test_header_declares_the_expected_calls():
    names = declared_functions()
    for must in ["pichol_cv", "pichol_exact_cv", "pichol_potrf_shifted_batched",
                 "pichol_fit", "pichol_eval", "pichol_solve_interp",
                 "pichol_solve_factors", "pichol_holdout", "pichol_gram"]:
        assert must in names


# The calls that compute a step of the method, and the passage that defines
# each: every one must cite a section, algorithm, table or theorem of the
# paper in its comment block.
COMPUTE_CALLS = [
    "pichol_pack", "pichol_unpack", "pichol_gram",
    "pichol_potrf_shifted_batched", "pichol_fit", "pichol_eval",
    "pichol_solve_interp", "pichol_solve_factors", "pichol_holdout",
    "pichol_holdout_direct", "pichol_slab_to_weights", "pichol_cv_gram",
    "pichol_cv_interp", "pichol_cv_exact", "pichol_cv_interp_grad",
    "pichol_cv_exact_grad", "pichol_cv_pinrmse", "pichol_cv", "pichol_exact_cv",
    "pichol_vectorize", "pichol_fit_vec", "pichol_eval_vec", "pichol_cv_batch",
    "pichol_factor_nrmse", "pichol_holdout_nrmse",
]
CITATION = re.compile(r"(Sec\.\s*\d|Algorithm\s*\d|Table\s*\d|Thm\.\s*\d)")


def comment_blocks():
    """name -> the comment block documenting it: the block right above its
    declaration, or above the run of declarations it belongs to."""
    text = open(HEADER).read()
    out = {}
    last = ""
    tok = re.compile(r"/\*.*?\*/|\b(pichol_[a-z_0-9]+)\s*\(|;|\{|\}", re.S)
    pending = ""
    for m in tok.finditer(text):
        t = m.group(0)
        if t.startswith("/*"):
            pending = t
        elif m.group(1):
            name = m.group(1)
            if pending:
                last = pending
                pending = ""
            out.setdefault(name, last)
    return out


def test_compute_calls_cite_the_paper():
    blocks = comment_blocks()
    missing = [n for n in COMPUTE_CALLS
               if n not in blocks or not CITATION.search(blocks[n])]
    assert not missing, "no passage of the paper cited for: %s" % missing


def test_citation_check_would_catch_a_missing_citation():
    assert not CITATION.search("/* Copy slabs to the weight layout. */")
    assert CITATION.search("/* Algorithm 1 steps 2-6 */")
    assert CITATION.search("/* (Sec. 3.1) */")


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name


def test_binding_covers_the_header():
    assert sorted(B.EXPORTED) == declared_functions()


def test_layout_arithmetic(lib):
    assert B.pichol_packed_elems(0) == 0
    assert B.pichol_packed_elems(1) == 128 * 128
    assert B.pichol_packed_elems(128) == 128 * 128
    assert B.pichol_packed_elems(129) == 3 * 128 * 128
    assert B.pichol_packed_elems(4096) == 32 * 33 // 2 * 128 * 128
    assert B.pichol_padded_order(300) == 384
    assert B.pichol_slab_cols(64, 10) == 640
    assert B.pichol_slab_cols(31, 10) == 384
    assert B.pichol_slab_cols(1, 1) == 128


def test_workspace_size_and_argument_checks(lib):
    p = B.make_problem(60000, 4096, 10, 5, g=6, r=2, q=64)
    wi = B.pichol_workspace_size(p, B.PICHOL_METHOD_INTERP)
    we = B.pichol_workspace_size(p, B.PICHOL_METHOD_EXACT)
    both = B.pichol_workspace_size(p, B.PICHOL_METHOD_INTERP | B.PICHOL_METHOD_EXACT)
    assert both == max(wi, we)
    S = B.pichol_packed_elems(4096)
    assert wi > 5 * 6 * S * 8 and we > 5 * 64 * S * 8
    for bad in [dict(r=6, g=6), dict(k=1), dict(k=65), dict(g=33), dict(r=8, g=9),
                dict(q=0), dict(precision=2), dict(precision=-1), dict(refine=-1),
                dict(refine=B.PICHOL_MAX_REFINE + 1), dict(basis=2), dict(basis=-1)]:
        kw = dict(g=6, r=2, q=64, k=5)
        kw.update(bad)
        k = kw.pop("k")
        p = B.make_problem(60000, 4096, 10, k, **kw)
        with pytest.raises(B.PicholError) as e:
            B.pichol_workspace_size(p, B.PICHOL_METHOD_INTERP)
        assert e.value.status == B.PICHOL_ERR_ARG
    p = B.make_problem(100, 10, 2, 5, g=3, r=2, q=4, ldx=9)  # ldx < d
    with pytest.raises(B.PicholError):
        B.pichol_workspace_size(p, B.PICHOL_METHOD_EXACT)


def test_problem_struct_layout():
    # int64 n, d, c; int32 k, g, r, q, normalize, precision, refine, basis;
    # int64 ldx, ldy
    assert ctypes.sizeof(B.Problem) == 3 * 8 + 8 * 4 + 2 * 8
    assert B.Problem.ldx.offset == 56
    p = B.make_problem(10, 3, 2, 2, precision=B.PICHOL_PREC_MIXED, refine=3, basis=1)
    assert p.precision == 1 and p.refine == 3 and p.basis == 1
    assert p.ldx == 3 and p.ldy == 2
    text = open(HEADER).read()
    assert "#define PICHOL_MAX_REFINE %d" % B.PICHOL_MAX_REFINE in text


def test_refine_grows_the_workspace(lib):
    p0 = B.make_problem(60000, 4096, 10, 5, g=6, r=2, q=64)
    p2 = B.make_problem(60000, 4096, 10, 5, g=6, r=2, q=64, refine=2)
    for m in [B.PICHOL_METHOD_INTERP, B.PICHOL_METHOD_EXACT]:
        extra = B.pichol_workspace_size(p2, m) - B.pichol_workspace_size(p0, m)
        # full-tile H_f and one correction slab per fold
        assert extra >= 5 * 4096 * 4096 * 8 + 5 * 4096 * 640 * 8


def test_status_strings(lib):
    for s in [0, -1, -2, -3, -4, -5]:
        assert lib.pichol_status_string(s)


def test_options(lib):
    assert B.pichol_get_option(B.PICHOL_OPT_LOOKAHEAD) == 0
    B.pichol_set_option(B.PICHOL_OPT_LOOKAHEAD, 1)
    assert B.pichol_get_option(B.PICHOL_OPT_LOOKAHEAD) == 1
    B.pichol_set_option(B.PICHOL_OPT_LOOKAHEAD, 0)
    with pytest.raises(B.PicholError):
        B.pichol_set_option(B.PICHOL_OPT_LOOKAHEAD, 7)
    with pytest.raises(B.PicholError):
        B.pichol_set_option(99, 0)
    assert B.pichol_get_option(99) == -1
    assert B.pichol_get_option(B.PICHOL_OPT_PANEL_GROUP) == 4
    for gsz in [1, 3, 8, 4]:
        B.pichol_set_option(B.PICHOL_OPT_PANEL_GROUP, gsz)
        assert B.pichol_get_option(B.PICHOL_OPT_PANEL_GROUP) == gsz
    for bad in [0, 9]:
        with pytest.raises(B.PicholError):
            B.pichol_set_option(B.PICHOL_OPT_PANEL_GROUP, bad)
    assert B.pichol_get_option(B.PICHOL_OPT_SOLVE_FORM) == 0
    for form in [1, 2, 0]:
        B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, form)
        assert B.pichol_get_option(B.PICHOL_OPT_SOLVE_FORM) == form
    for bad in [-1, 3]:
        with pytest.raises(B.PicholError):
            B.pichol_set_option(B.PICHOL_OPT_SOLVE_FORM, bad)


def test_batch_tuning_struct_layout():
    t = B.BatchTuning()
    assert ctypes.sizeof(t) == 4 * (2 + 32 + 32)
    assert B.BatchTuning.solve_form.offset == 4 * (2 + 32)
    text = open(HEADER).read()
    assert "int32_t solve_form[32];" in text


def test_noalloc_holdout_rejects_oversize_before_touching_the_device(lib):
    """The allocation-free hold-out call checks its scratch limit on the host
    first: at d = 4096, q = 64, c = 10 the partial sums of 13 folds exceed
    16 MiB.  (Nothing is enqueued, so no GPU is needed.)"""
    assert B.pichol_holdout_workspace(4096, 13, 64, 10) > B.PICHOL_HOLDOUT_SCRATCH_BYTES
    assert B.pichol_holdout_workspace(4096, 12, 64, 10) <= B.PICHOL_HOLDOUT_SCRATCH_BYTES
    fake = ctypes.c_void_p(256)  # never dereferenced: the call returns first
    nv = (ctypes.c_int64 * 13)(*([12000] * 13))
    st = lib.pichol_holdout_noalloc(4096, 13, 10, 64, fake, fake, fake, fake,
                                    ctypes.cast(nv, ctypes.c_void_p), fake, fake,
                                    None)
    assert st == B.PICHOL_ERR_WORKSPACE
    assert b"static scratch" in lib.pichol_last_error()
    assert "#define PICHOL_HOLDOUT_SCRATCH_BYTES (16u << 20)" in open(HEADER).read()
    assert B.PICHOL_HOLDOUT_SCRATCH_BYTES == 16 << 20
