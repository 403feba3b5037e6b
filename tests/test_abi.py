"""The C-ABI library loads, exports every declared entry point, and rejects
malformed systems before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polyeval.h")
LIB = os.path.join(ROOT, "paper_1402_2626_amd", "libpolyeval.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pe_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpolyeval.so is not built (python -m paper_1402_2626_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_interface():
    names = declared_functions()
    for must in ("pe_system_create", "pe_eval", "pe_eval_adjoint", "pe_batch_eval", "pe_newton_step",
                 "pe_autotune", "pe_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_1402_2626_amd import polyeval
    assert set(polyeval.SIGNATURES) == set(declared_functions())
    assert polyeval.abi_version() == 1


def _create(lib, level, n, poly_ptr, mon_ptr, var_idx, exps, coef):
    lib.pe_system_create.restype = ctypes.c_int32
    lib.pe_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    arrs = [np.ascontiguousarray(a, dtype=dt) for a, dt in
            ((poly_ptr, np.int64), (mon_ptr, np.int64), (var_idx, np.int32), (exps, np.int32), (coef, np.float64))]
    st = lib.pe_system_create(ctypes.byref(h), ctypes.c_int32(level), ctypes.c_int32(n),
                              ctypes.c_int32(len(poly_ptr) - 1), *[ctypes.c_void_p(a.ctypes.data) for a in arrs],
                              ctypes.c_void_p(None))
    return st, h, lib.pe_last_error().decode()


GOOD = dict(level=2, n=4, poly_ptr=[0, 2], mon_ptr=[0, 2, 3], var_idx=[0, 3, 1], exps=[1, 2, 3],
            coef=np.zeros((2, 2, 2)))


@pytest.mark.parametrize("change, status, words", [
    (dict(level=3), -1, "level"),
    (dict(level=16 | 2), -1, "level"),
    (dict(level=8 | 3), -1, "level"),
    (dict(level=8 | 2, var_idx=[0, 4, 1]), -1, "out of range"),
    (dict(n=0), -1, "n_vars"),
    (dict(n=70000), -3, "65535"),
    (dict(var_idx=[0, 4, 1]), -1, "out of range"),
    (dict(var_idx=[0, -1, 1]), -1, "out of range"),
    (dict(exps=[1, 0, 3]), -1, "exponent"),
    (dict(exps=[1, 70000, 3]), -1, "exponent"),
    (dict(var_idx=[2, 2, 1]), -1, "duplicate"),
    (dict(mon_ptr=[0, 3, 2]), -1, "nondecreasing"),
    (dict(poly_ptr=[1, 2]), -1, "poly_ptr"),
    (dict(mon_ptr=[0, 1025, 1026], var_idx=list(range(1025)) + [0], exps=[1] * 1026, n=2000), -3, "1024"),
])
def test_validation_errors(lib, change, status, words):
    args = dict(GOOD)
    args.update(change)
    st, h, msg = _create(lib, args["level"], args["n"], args["poly_ptr"], args["mon_ptr"], args["var_idx"],
                         args["exps"], args["coef"])
    assert st == status, msg
    assert words in msg
    assert not h.value


def test_lstsq_level_codes(lib):
    """pe_lstsq takes the level codes 1, 2, 4 and PE_REAL | 1, 2, 4; other
    codes are refused before any device work (workspace size 0, PE_EINVAL)."""
    lib.pe_lstsq_workspace_bytes.restype = ctypes.c_size_t
    lib.pe_lstsq.restype = ctypes.c_int32
    for code in (1, 2, 4, 9, 10, 12):
        assert lib.pe_lstsq_workspace_bytes(code, 1, 10, 5) > 0
    for code in (0, 3, 8, 11, 18):
        assert lib.pe_lstsq_workspace_bytes(code, 1, 10, 5) == 0
        assert lib.pe_lstsq(code, 1, 10, 5, None, None, None, None, None, None, None) == -1
    # real workspaces are smaller than complex ones (one component)
    assert lib.pe_lstsq_workspace_bytes(10, 1, 100, 50) < lib.pe_lstsq_workspace_bytes(2, 1, 100, 50)


def test_null_arguments(lib):
    lib.pe_eval.restype = ctypes.c_int32
    assert lib.pe_eval(None, 1, None, None, None, None) == -1
    lib.pe_system_destroy.restype = ctypes.c_int32
    assert lib.pe_system_destroy(None) == 0
