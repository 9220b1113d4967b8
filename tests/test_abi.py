"""The C-ABI library loads and exports every entry point include/dngd.h
declares (no compute: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dngd.h")
LIB = os.path.join(ROOT, "paper_2505_21404_amd", "libdngd.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dngd_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("dngd_residual_jacobian", "dngd_gram", "dngd_cholesky_solve",
                     "dngd_nystrom_pcg", "dngd_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdngd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.dngd_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.dngd_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdngd.so not built")
def test_binding_covers_every_export():
    from paper_2505_21404_amd import dngd
    assert sorted(dngd.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdngd.so not built")
def test_argument_validation_without_gpu():
    """Invalid arguments are rejected on the host before anything is enqueued."""
    from paper_2505_21404_amd import dngd
    lib = dngd._lib
    d = dngd.ProblemDesc()
    d.pde, d.n_layers = 0, 0
    h = ctypes.c_void_p()
    assert lib.dngd_problem_create(ctypes.byref(d), ctypes.byref(h)) == dngd.EINVAL
    assert b"n_layers" in lib.dngd_last_error()
    # dngd_gram: ldJ < n
    assert lib.dngd_gram(10, 20, ctypes.c_void_p(8), 10, 0, 1, 0.0, ctypes.c_void_p(8), 10,
                         None) == dngd.EINVAL
    # passes must be 1 or 3 for FP32 J
    assert lib.dngd_gram(10, 20, ctypes.c_void_p(8), 20, 1, 2, 0.0, ctypes.c_void_p(8), 10,
                         None) == dngd.EINVAL
    info = ctypes.c_int64()
    assert lib.dngd_cholesky_solve(0, ctypes.c_void_p(8), 1, 0, 0, None, 1, ctypes.byref(info),
                                   None) == dngd.EINVAL
    # the allocation-free variant rejects m beyond its static scratch (m <= 2048)
    assert lib.dngd_cholesky_solve_noalloc(2049, ctypes.c_void_p(8), 2049, 0, 1,
                                           ctypes.c_void_p(8), 2049, ctypes.byref(info),
                                           None) == dngd.EINVAL
    assert b"2048" in lib.dngd_last_error()
    # the refined solve: a refinement description is required and checked
    K, B = ctypes.c_void_p(256), ctypes.c_void_p(256)
    assert lib.dngd_cholesky_solve_refine(4, K, 4, 0, 1, B, 4, None, None, ctypes.byref(info),
                                          None) == dngd.EINVAL
    good = dict(J=256, n=8, ldJ=8, j_dtype=dngd.F32, sweeps=2, lam=1e-3)
    for change, word in ((dict(J=None), b"null"), (dict(J=264), b"aligned"),
                         (dict(ldJ=6), b"ldJ"), (dict(n=0), b"n >= 1"),
                         (dict(j_dtype=dngd.BF16), b"j_dtype"), (dict(sweeps=17), b"sweeps"),
                         (dict(lam=float("nan")), b"lambda")):
        R = dngd.Refine(**{**good, **change})
        assert lib.dngd_cholesky_solve_refine(4, K, 4, 0, 1, B, 4, ctypes.byref(R), None,
                                              ctypes.byref(info), None) == dngd.EINVAL, change
        assert word in lib.dngd_last_error(), (change, lib.dngd_last_error())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdngd.so not built")
def test_description_validation_and_defaults_without_gpu():
    """dngd_footprint_desc validates a description on the host; the step
    options have the documented defaults."""
    from paper_2505_21404_amd import dngd
    import workloads as W
    ok = W.config(0)
    assert dngd.footprint_of(ok.pde, ok.widths, ok.n_int, ok.n_bdy, ok.n_init) > 0
    bad = [
        (dngd.POISSON, [2, 8, 2], 10, 5, 0),         # two outputs
        (dngd.POISSON, [9, 8, 1], 10, 5, 0),         # d_in above 8
        (dngd.POISSON, [2, 8, 1], 10, 5, 3),         # initial points without heat
        (dngd.HEAT, [1, 8, 1], 10, 5, 3),            # heat needs time plus space
        (dngd.POISSON, [2, 5000, 1], 10, 5, 0),      # hidden width above 4096
        (dngd.POISSON, [2, 8, 1], 0, 0, 0),          # no points
        (dngd.POISSON, [2, 8, 1], -1, 5, 0),         # negative count
    ]
    for pde, widths, ni, nb, n0 in bad:
        with pytest.raises(dngd.DngdError) as e:
            dngd.footprint_of(pde, widths, ni, nb, n0)
        assert e.value.status == dngd.EINVAL
    o = dngd.StepOpts()
    dngd._lib.dngd_step_opts_default(ctypes.byref(o))
    assert (o.precision, o.solver, o.ga, o.ir_sweeps, o.gram_passes) == (dngd.MIXED, dngd.DENSE, 1, 2, 0)
    assert o.eps_norm == 0.0 and o.pcg_tol == 1e-6 and o.pcg_maxit == 500 and o.ir_tol == 1e-5
    assert o.no_lookahead == 0 and not o.alpha_out and not o.fvv_out
