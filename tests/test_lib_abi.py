"""The C-ABI library loads and exports every entry point declared in include/skrylov.h.

Host-only checks (no GPU): symbol table, parameter defaults and layout, and the CSR
validation that runs on the host before any device work.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2311_16019_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "skrylov.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SKR_API\s+(?:const\s+char\s*\*|int)\s+(skr_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("skr_op_create_csr", "skr_solve", "skr_adjoint_solve", "skr_true_residual", "skr_pairing_grads"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature"
    assert set(_lib.SIGNATURES) == set(declared_symbols())


def test_params_default_and_layout():
    lib = _lib.load()
    p = _lib.Params()
    assert lib.skr_params_default(ctypes.byref(p)) == 0
    assert ctypes.sizeof(p) == 72
    assert (p.k, p.maxit, p.p, p.zeta, p.s) == (2, 200, 20, 8, 0)
    assert p.tol == 1e-6 and p.trunc_tol == 1e-12 and p.precision == _lib.SKR_FP64
    assert p.orth == _lib.SKR_ORTH_EUCLIDEAN
    assert lib.skr_params_default(None) == _lib.SKR_EINVAL
    assert lib.skr_version().decode().startswith("skrylov")


def _create(n, rowptr, colind, vals):
    lib = _lib.load()
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colind, dtype=np.int32)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    h = ctypes.c_void_p()
    code = lib.skr_op_create_csr(n, int(rp[-1]), rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p),
                                 v.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.byref(h))
    return code, lib.skr_last_error().decode()


@pytest.mark.parametrize("rowptr,colind,msg", [
    ([0, 1, 3], [0, 5, 1], "column index out of range"),
    ([0, 2, 1], [0, 1], "nondecreasing"),
    ([1, 2, 3], [0, 1, 0], "start at 0"),
    ([0, 1, 2], [0, -1], "column index out of range"),
])
def test_malformed_csr_is_rejected_on_the_host(rowptr, colind, msg):
    code, err = _create(2, rowptr, colind, np.ones(len(colind)))
    assert code == _lib.SKR_EINVAL
    assert msg in err


def test_null_arguments_are_errors():
    lib = _lib.load()
    assert lib.skr_solve(None, None, None, None, 1, None, None, None) == _lib.SKR_EINVAL
    assert lib.skr_result_info(None, None, None, None, None) == _lib.SKR_EINVAL
    assert lib.skr_op_size(None, None, None) == _lib.SKR_EINVAL
