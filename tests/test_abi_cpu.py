"""Host-side checks of the C-ABI library (no GPU): it loads, exports every entry point
the header declares, and its pure host calls behave."""
import ctypes
import os

import pytest

from paper_1301_5914_amd import hobi


def test_library_exports_every_declared_symbol():
    lib = hobi.lib()
    declared = hobi.header_symbols()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name


def test_params_default():
    p = hobi.hobi_params_default()
    assert (p.eps1, p.eps2, p.kappa, p.rtol) == (1.0, 80.0, 0.1257, 1e-6)
    assert (p.max_iter, p.restart, p.precision, p.method, p.diag_scaling) == (200, 200, hobi.HOBI_FP64, 0, 2)
    assert p.tree_refine == 0
    assert (p.tree_theta, p.tree_degree, p.tree_leaf, p.tree_batch) == (0.0, 5, 256, 128)


def test_null_arguments_are_rejected_without_touching_a_device():
    lib = hobi.lib()
    out = ctypes.c_void_p()
    assert lib.hobi_ctx_create(0, None, None) == 1            # HOBI_E_ARG
    assert lib.hobi_problem_create(None, 0, None, None, 0, None, 0, None, None, None,
                                   ctypes.byref(out)) == 1
    assert lib.hobi_matvec(None, None, None, 0) == 1
    assert lib.hobi_solve(None, None, None, None, None) == 1
    assert lib.hobi_field(None, None, 0, 0, None, None, None, None, None, None) == 1
    assert lib.hobi_last_error(None) == b"null context"


def test_header_documents_status_codes():
    text = open(hobi.HEADER).read()
    for name in hobi.STATUS.values():
        assert name in text


def test_built_for_gfx950():
    blob = open(hobi.LIB_PATH, "rb").read()
    assert b"gfx950" in blob
