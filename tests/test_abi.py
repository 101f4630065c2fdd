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
    assert L.cmc_pair_cells(1, None, None, None, None, None, None, None, 1, 0, 1, None, None, None,
                            None, None) == 1
    assert L.cmc_collide_step(None, None, None, None, None, None, None, None, None, None, 0, None) == 1
    assert L.cmc_expected_yield(None, 1, *([None] * 4), 0, *([None] * 4), 1e-16, 0, None, None, None, None) == 1
    # the expected-yield calls check their arguments before touching the
    # tables (a placeholder handle is never dereferenced): no cell is a
    # no-op with NULL arrays; cells need every array; dt and the precision
    # are checked either way
    t = C.c_void_p(1)
    assert L.cmc_expected_yield(t, 0, *([None] * 4), 0, *([None] * 4), 1e-16, 0, None, None, None, None) == 0
    assert L.cmc_expected_yield_backward(t, 0, *([None] * 4), 0, *([None] * 4), 1e-16, 1, *([None] * 8), None, None) == 0
    assert L.cmc_expected_yield(t, 2, *([None] * 4), 0, *([None] * 4), 1e-16, 0, None, None, None, None) == 1
    assert b"NULL cell array" in L.cmc_last_error()
    # cells with particles need the particle arrays; n_part < 0 is refused
    assert L.cmc_expected_yield(t, 2, *([C.c_void_p(8)] * 4), 3, *([None] * 4), 1e-16, 0, None, None,
                                None, None) == 1
    assert b"NULL particle array" in L.cmc_last_error()
    assert L.cmc_expected_yield(t, 0, *([None] * 4), -1, *([None] * 4), 1e-16, 0, None, None, None,
                                None) == 1
    assert b"n_part" in L.cmc_last_error()
    assert L.cmc_expected_yield_backward(t, 2, *([None] * 4), 0, *([None] * 4), 1e-16, 0, *([None] * 8), None, None) == 1
    assert L.cmc_expected_yield(t, 0, *([None] * 4), 0, *([None] * 4), 0.0, 0, None, None, None, None) == 1
    assert b"dt" in L.cmc_last_error()
    assert L.cmc_expected_yield(t, 0, *([None] * 4), 0, *([None] * 4), 1e-16, 7, None, None, None, None) == 1
    assert b"precision" in L.cmc_last_error()
    assert L.cmc_expected_yield(t, -1, *([None] * 4), 0, *([None] * 4), 1e-16, 0, None, None, None, None) == 1
    assert L.cmc_tables_size(None, 0) == -1
    assert L.cmc_tables_free(None) == 0
    # the no-allocation step: its static workspace bounds the cells, checked
    # before any device call
    assert L.cmc_noalloc_max_cells() == 16384
    big = cmc._Cells(16385, None, None, None, None)
    prm = cmc._StepParams(1e-16, 1, 0, 1, 0, 0, 1, 1e-6)
    assert L.cmc_collide_step_noalloc(None, C.byref(big), None, None, None, None, None, C.byref(prm), None,
                                      None) == 2
    assert b"16384" in L.cmc_last_error()
    assert L.cmc_collide_step_noalloc(None, None, None, None, None, None, None, None, None, None) == 1


def test_binding_rejects_wrong_element_types():
    # the binding checks the element type the C ABI reads before anything
    # else (here on host tensors, so the first array of each call is the
    # wrong one): float32 where doubles are read, int32 offsets
    import pytest
    import torch
    import paper_1907_02814_amd as cmc
    f4 = torch.zeros(4, dtype=torch.float32)
    f8 = torch.zeros(4, dtype=torch.float64)
    off32 = torch.zeros(3, dtype=torch.int32)
    off64 = torch.zeros(3, dtype=torch.int64)

    class T:
        handle = None
    with pytest.raises(TypeError, match="float64"):
        cmc.expected_yield(T(), f4[:2], f8[:2], f8[:2], off64, f8, f8, f8, f8, 1e-16)
    with pytest.raises(TypeError, match="float64"):
        cmc.expected_yield_backward(T(), f4[:2], f8[:2], f8[:2], off64, f8, f8, f8, f8, 1e-16, f8[:2])
    with pytest.raises(TypeError, match="int64"):
        cmc.pair_cells(off32, off32[:2], off64, off32[:2], f8, f8, 1, 0, 1, off64)
    with pytest.raises(TypeError, match="int64"):
        cmc._species({"off": off32, "px": f8, "py": f8, "pz": f8, "w": f8})
    with pytest.raises(TypeError, match="int32"):
        cmc._species({"off": off64.cuda() if torch.cuda.is_available() else None, "count": off64})


def test_binding_rejects_inconsistent_lengths():
    import pytest
    import torch
    import paper_1907_02814_amd as cmc
    f8 = torch.zeros(4, dtype=torch.float64)
    off = torch.zeros(3, dtype=torch.int64)

    class T:
        handle = None
    with pytest.raises(ValueError, match="cells"):
        cmc.expected_yield(T(), f8[:2], f8[:3], f8[:2], off, f8, f8, f8, f8, 1e-16)
    with pytest.raises(ValueError, match="off"):
        cmc.expected_yield(T(), f8[:2], f8[:2], f8[:2], off[:2], f8, f8, f8, f8, 1e-16)
    with pytest.raises(ValueError, match="electrons"):
        cmc.expected_yield(T(), f8[:2], f8[:2], f8[:2], off, f8, f8[:3], f8, f8, 1e-16)
    with pytest.raises(ValueError, match="cells"):
        cmc.expected_yield_backward(T(), f8[:2], f8[:2], f8[:2], off, f8, f8, f8, f8, 1e-16, f8[:3])
    cnt = torch.zeros(2, dtype=torch.int32)
    with pytest.raises(ValueError, match="offsets"):
        cmc.pair_cells(off, cnt, off[:2], cnt, f8, f8, 1, 0, 1, off)
    with pytest.raises(ValueError, match="cell_id"):
        cmc.pair_cells(off, cnt, off, cnt, f8, f8, 1, 0, 1, off, cell_id=off)


def test_binding_rejects_bad_yield_offsets():
    # offsets that decrease, do not start at 0 or pass the end of the
    # electron arrays are refused before any launch (the kernels check
    # every cell again on the device)
    import pytest
    import torch
    import paper_1907_02814_amd as cmc
    f8 = torch.zeros(4, dtype=torch.float64)

    class T:
        handle = None
    for bad in ([0, 3, 2], [1, 2, 4], [0, 2, 5]):
        off = torch.tensor(bad, dtype=torch.int64)
        with pytest.raises(ValueError, match="non-decreasing"):
            cmc.expected_yield(T(), f8[:2], f8[:2], f8[:2], off, f8, f8, f8, f8, 1e-16)
        with pytest.raises(ValueError, match="non-decreasing"):
            cmc.expected_yield_backward(T(), f8[:2], f8[:2], f8[:2], off, f8, f8, f8, f8, 1e-16, f8[:2])


def test_missing_library_fails_loudly():
    # no fallback: without the built HIP library every call raises
    import pytest
    import paper_1907_02814_amd as cmc
    saved_path, saved_lib = cmc.LIB_PATH, cmc._LIB
    try:
        cmc.LIB_PATH, cmc._LIB = "/nonexistent/libcmc.so", None
        with pytest.raises(ImportError, match="not built"):
            cmc.get_lib()
        with pytest.raises(ImportError):
            cmc.build_tables(29)
    finally:
        cmc.LIB_PATH, cmc._LIB = saved_path, saved_lib


def test_screening_calls_check_arguments_without_gpu():
    """cmc_screening_functions / cmc_cross_sections: the handle, the form,
    the process and n are checked on the host; n = 0 is a no-op with NULL
    arrays (a placeholder handle is never dereferenced before that)."""
    import paper_1907_02814_amd as cmc
    L = cmc.get_lib()
    t = C.c_void_p(1)
    assert L.cmc_screening_functions(None, 0, 4, *([None] * 8)) == 1
    assert b"tables is NULL" in L.cmc_last_error()
    assert L.cmc_screening_functions(t, 2, 4, *([None] * 8)) == 1
    assert b"unknown form" in L.cmc_last_error()
    assert L.cmc_screening_functions(t, 1, -1, *([None] * 8)) == 1
    assert L.cmc_screening_functions(t, 1, 0, *([None] * 8)) == 0
    assert L.cmc_screening_functions(t, 1, 3, *([None] * 8)) == 1
    assert b"NULL array" in L.cmc_last_error()
    assert L.cmc_cross_sections(t, cmc.TRIDENT, 0, 0, *([None] * 8)) == 1
    assert b"process" in L.cmc_last_error()
    assert L.cmc_cross_sections(t, cmc.BH, 5, 0, *([None] * 8)) == 1
    assert L.cmc_cross_sections(t, cmc.BREMS, 1, 0, *([None] * 8)) == 0
    assert L.cmc_cross_sections(t, cmc.BREMS, 1, 2, *([None] * 8)) == 1


def test_misaligned_arrays_are_refused_on_the_host():
    """A device array pointer that is not aligned to its element type is
    refused before anything is launched (the pointers here are placeholders,
    never dereferenced; each call also lacks what a launch would need, so
    nothing could run if a check were missing)."""
    import paper_1907_02814_amd as cmc
    L = cmc.get_lib()
    ok8, odd = C.c_void_p(1 << 20), C.c_void_p((1 << 20) + 4)
    t = C.c_void_p(1)
    # collide_step: a cell array, then a species array (workspace NULL)
    cells = cmc._Cells(2, odd, ok8, ok8, None)
    tal = cmc._Tallies(ok8, ok8, ok8)
    P = cmc._StepParams()
    P.dt, P.processes, P.precision, P.schedule, P.max_per_cell, P.near_rel = 1e-16, 1, 0, 2, 64, 1e-6
    sp = cmc._Species(ok8, ok8, ok8, ok8, ok8, ok8, None)
    args = [C.byref(sp)] * 5
    assert L.cmc_collide_step(t, C.byref(cells), *args, C.byref(P), C.byref(tal), None, 0, None) == 1
    assert b"aligned" in L.cmc_last_error()
    cells = cmc._Cells(2, ok8, ok8, ok8, None)
    bad = cmc._Species(ok8, ok8, odd, ok8, ok8, ok8, None)
    assert L.cmc_collide_step(t, C.byref(cells), C.byref(bad), *args[1:], C.byref(P), C.byref(tal), None, 0,
                              None) == 1
    assert b"aligned" in L.cmc_last_error() and b"electrons" in L.cmc_last_error()
    bad = cmc._Species(ok8, C.c_void_p((1 << 20) + 2), ok8, ok8, ok8, ok8, None)   # count: int32
    assert L.cmc_collide_step(t, C.byref(cells), args[0], C.byref(bad), *args[2:], C.byref(P), C.byref(tal), None,
                              0, None) == 1
    assert b"aligned" in L.cmc_last_error() and b"photons" in L.cmc_last_error()
    # expected yield: the offsets (Y NULL)
    assert L.cmc_expected_yield(t, 2, ok8, ok8, ok8, odd, 4, ok8, ok8, ok8, ok8, 1e-16, 0, None, None, None,
                                None) == 1
    assert b"aligned" in L.cmc_last_error()
    # pair_cells: a pair array (int32) at an odd address (no stream, no tables: a
    # missing check would reach the launch, which fails without a GPU)
    odd2 = C.c_void_p((1 << 20) + 2)
    assert L.cmc_pair_cells(1, None, ok8, None, ok8, None, ok8, ok8, 1, 0, 1, ok8, odd2, ok8, None, None) == 1
    assert b"aligned" in L.cmc_last_error()
