"""The C ABI library loads and exports every symbol include/cmc.h declares;
host-side argument checks answer without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cmc_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1907_02814_amd as cmc
    L = cmc.get_lib()
    declared = _declared()
    assert declared, "no declarations found"
    assert set(declared) == set(cmc.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_host_argument_errors_without_gpu():
    import paper_1907_02814_amd as cmc
    L = cmc.get_lib()
    h = C.c_void_p()
    assert L.cmc_build_tables(0, None, C.byref(h)) == 1
    assert b"Z = 0" in L.cmc_last_error()
    assert L.cmc_build_tables(101, None, C.byref(h)) == 1
    assert L.cmc_build_tables(29, None, None) == 1
    assert L.cmc_pair_cells(1, None, None, None, None, None, None, 1, 0, 1, None, None, None, None,
                            None) == 1
    assert L.cmc_collide_step(None, None, None, None, None, None, None, None, None, None, 0, None) == 1
    assert L.cmc_expected_yield(None, 1, *([None] * 8), 1e-16, 0, None, None, None) == 1
    # the expected-yield calls check their arguments before touching the
    # tables (a placeholder handle is never dereferenced): no cell is a
    # no-op with NULL arrays; cells need every array; dt and the precision
    # are checked either way
    t = C.c_void_p(1)
    assert L.cmc_expected_yield(t, 0, *([None] * 8), 1e-16, 0, None, None, None) == 0
    assert L.cmc_expected_yield_backward(t, 0, *([None] * 8), 1e-16, 1, *([None] * 8), None) == 0
    assert L.cmc_expected_yield(t, 2, *([None] * 8), 1e-16, 0, None, None, None) == 1
    assert b"NULL array" in L.cmc_last_error()
    assert L.cmc_expected_yield_backward(t, 2, *([None] * 8), 1e-16, 0, *([None] * 8), None) == 1
    assert L.cmc_expected_yield(t, 0, *([None] * 8), 0.0, 0, None, None, None) == 1
    assert b"dt" in L.cmc_last_error()
    assert L.cmc_expected_yield(t, 0, *([None] * 8), 1e-16, 7, None, None, None) == 1
    assert b"precision" in L.cmc_last_error()
    assert L.cmc_expected_yield(t, -1, *([None] * 8), 1e-16, 0, None, None, None) == 1
    assert L.cmc_tables_size(None, 0) == -1
    assert L.cmc_tables_free(None) == 0
