"""cmc: pairwise Coulomb-process Monte Carlo (Bremsstrahlung, Bethe-Heitler,
Trident) for weighted PIC macro-particles on MI355X.

A thin ctypes binding of libcmc.so (include/cmc.h): every function here only
marshals torch tensors (device memory) and the current HIP stream into the
C ABI; all work runs in the library's HIP kernels.  The first call into the
library fails loudly (ImportError) when libcmc.so has not been built; there
is no fallback path.

Paper: Martinez et al., "High-Energy Radiation and Pair Production by Coulomb
Processes in Particle-In-Cell Simulations" (arXiv:1907.02814).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcmc.so")

BREMS, BH, TRIDENT = 1, 2, 4
FP64, FP32 = 0, 1
SCHED_AUTO, SCHED_CELL, SCHED_GROUP, SCHED_WAVE, SCHED_HYBRID, SCHED_QUEUE, SCHED_SPLIT = 0, 1, 2, 3, 4, 5, 6
SCHED_NO_STREAM = 0x100   # OR-ed into a schedule: no stream kernel
SCREEN_REDUCED, SCREEN_TFD = 0, 1
MAX_PER_CELL = 16384
ST_OVERFLOW, ST_GAMMA_HIGH, ST_BAD_CELL, ST_BAD_WEIGHT, ST_TOO_LARGE, ST_BAD_OFFSETS = 1, 2, 4, 8, 16, 32
I_NAMES = ["pairs_br", "pairs_tr", "pairs_bh", "ev_br", "ev_tr", "ev_bh",
           "near_br", "near_tr", "near_bh", "drop_ph", "drop_el", "drop_po"]
D_NAMES = ["nab_ei", "nab_gi", "E_br", "E_tr", "E_bh", "dE_el", "dE_ph",
           "W_br", "W_tr", "W_bh"]
TABLE_NAMES = ["sigR", "skR", "cdfR", "sigU", "skU", "cdfU", "sigN", "skN", "cdfN",
               "sigB", "cdfB", "cdfT", "cdfS"]
EXPORTS = ["cmc_last_error", "cmc_build_tables", "cmc_tables_free", "cmc_tables_size",
           "cmc_tables_export", "cmc_pair_cells", "cmc_collide_step", "cmc_step_workspace_bytes",
           "cmc_expected_yield", "cmc_expected_yield_backward", "cmc_collide_step_noalloc",
           "cmc_noalloc_max_cells", "cmc_screening_functions", "cmc_cross_sections",
           "cmc_merge_species", "cmc_rebin_offsets", "cmc_rebin_copy"]

_vp = C.c_void_p
_i64 = C.c_int64


class CmcError(RuntimeError):
    pass


class _Cells(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("Zstar", _vp), ("n_i", _vp), ("T_e", _vp), ("cell_id", _vp)]


class _Species(C.Structure):
    _fields_ = [("off", _vp), ("count", _vp), ("px", _vp), ("py", _vp), ("pz", _vp),
                ("w", _vp), ("parent", _vp)]


class _StepParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("seed", C.c_uint64), ("step", C.c_uint64),
                ("processes", C.c_uint32), ("precision", C.c_int32), ("schedule", C.c_int32),
                ("max_per_cell", C.c_int32), ("near_rel", C.c_double), ("pass_events", _vp * 2),
                ("step_counter", _vp)]


class _Tallies(C.Structure):
    _fields_ = [("ti", _vp), ("td", _vp), ("status", _vp)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libcmc.so is not built ({LIB_PATH}); run "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    L.cmc_last_error.restype = C.c_char_p
    L.cmc_build_tables.argtypes = [C.c_int32, _vp, C.POINTER(_vp)]
    L.cmc_tables_free.argtypes = [_vp]
    L.cmc_tables_size.argtypes = [_vp, C.c_int32]
    L.cmc_tables_size.restype = _i64
    L.cmc_tables_export.argtypes = [_vp, C.c_int32, _vp, _i64]
    L.cmc_pair_cells.argtypes = [_i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_uint64, C.c_uint64,
                                 C.c_uint32, _vp, _vp, _vp, _vp, _vp]
    L.cmc_collide_step.argtypes = [_vp, C.POINTER(_Cells), C.POINTER(_Species), C.POINTER(_Species),
                                   C.POINTER(_Species), C.POINTER(_Species), C.POINTER(_Species),
                                   C.POINTER(_StepParams), C.POINTER(_Tallies), _vp, C.c_size_t, _vp]
    L.cmc_step_workspace_bytes.argtypes = [_i64, C.c_int32]
    L.cmc_step_workspace_bytes.restype = C.c_size_t
    L.cmc_collide_step_noalloc.argtypes = [_vp, C.POINTER(_Cells), C.POINTER(_Species), C.POINTER(_Species),
                                           C.POINTER(_Species), C.POINTER(_Species), C.POINTER(_Species),
                                           C.POINTER(_StepParams), C.POINTER(_Tallies), _vp]
    L.cmc_noalloc_max_cells.argtypes = []
    L.cmc_noalloc_max_cells.restype = C.c_size_t
    L.cmc_expected_yield.argtypes = ([_vp, _i64] + [_vp] * 4 + [_i64] + [_vp] * 4
                                     + [C.c_double, C.c_int32, _vp, _vp, _vp, _vp])
    L.cmc_expected_yield_backward.argtypes = ([_vp, _i64] + [_vp] * 4 + [_i64] + [_vp] * 4
                                              + [C.c_double, C.c_int32] + [_vp] * 8 + [_vp, _vp])
    L.cmc_merge_species.argtypes = [_i64, C.POINTER(_Species), C.POINTER(_Species), _vp, _vp, _vp]
    L.cmc_rebin_offsets.argtypes = [_i64, C.POINTER(_Species), C.c_int32, _vp, _vp]
    L.cmc_rebin_copy.argtypes = [_i64, C.POINTER(_Species), C.POINTER(_Species), _vp]
    L.cmc_screening_functions.argtypes = [_vp, C.c_int32, _i64] + [_vp] * 8
    L.cmc_cross_sections.argtypes = [_vp, C.c_int32, C.c_int32, _i64] + [_vp] * 8
    for name in ("cmc_build_tables", "cmc_tables_free", "cmc_tables_export", "cmc_pair_cells",
                 "cmc_collide_step", "cmc_expected_yield", "cmc_expected_yield_backward",
                 "cmc_collide_step_noalloc", "cmc_screening_functions", "cmc_cross_sections",
                 "cmc_merge_species", "cmc_rebin_offsets", "cmc_rebin_copy"):
        getattr(L, name).restype = C.c_int
    return L


_LIB = None


def get_lib():
    """The loaded libcmc.so (ImportError if it has not been built)."""
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


def __getattr__(name):
    if name == "lib":
        return get_lib()
    raise AttributeError(name)


def _check(rc: int, what: str):
    if rc != 0:
        msg = get_lib().cmc_last_error()
        raise CmcError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")


_PLACEHOLDER = {}


def _ptr(t, dtype=None) -> Optional[int]:
    """Device pointer of a contiguous tensor (None -> NULL) of the element
    type the C ABI reads there (`dtype`, a torch dtype name, checked when
    given).  An empty tensor (a species with no particles anywhere) gets a
    one-element placeholder so that required arrays are never NULL; the
    kernels never address it."""
    if t is None:
        return None
    if dtype is not None and str(t.dtype) != "torch." + dtype:
        raise TypeError(f"expected a {dtype} tensor, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    if not t.is_cuda:
        raise ValueError("tensors must be on the GPU")
    if t.numel() == 0:
        import torch
        key = (t.device, t.dtype)
        if key not in _PLACEHOLDER:
            _PLACEHOLDER[key] = torch.zeros(1, dtype=t.dtype, device=t.device)
        return _PLACEHOLDER[key].data_ptr()
    return t.data_ptr()


def _lengths(**groups):
    """Element counts that must agree (no device read): each keyword names
    a group as (expected count, tensors...)."""
    for name, (n, *ts) in groups.items():
        for t in ts:
            if t is not None and t.numel() != n:
                raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")


def _stream(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Tables:
    """Device tables for element Z (cmc_build_tables)."""

    def __init__(self, Z: int, stream=None):
        h = _vp()
        _check(get_lib().cmc_build_tables(int(Z), _stream(stream), C.byref(h)), "cmc_build_tables")
        self.Z = int(Z)
        self._h = h

    @property
    def handle(self):
        return self._h

    def export(self, name) -> np.ndarray:
        which = TABLE_NAMES.index(name) if isinstance(name, str) else int(name)
        n = get_lib().cmc_tables_size(self._h, which)
        out = np.zeros(n)
        _check(get_lib().cmc_tables_export(self._h, which, out.ctypes.data, n), "cmc_tables_export")
        return out

    def close(self):
        if getattr(self, "_h", None):
            get_lib().cmc_tables_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_tables(Z: int, stream=None) -> Tables:
    return Tables(Z, stream)


def pair_cells(a_off, a_cnt, b_off, b_cnt, wa, wb, seed, step, pass_, pair_off, stream=None, cell_id=None):
    """Pair indices of every cell (cmc_pair_cells); returns (pa, pb, n_ab).
    cell_id: int64 global cell indices keying the draws (None = position)."""
    import torch
    n_cells = a_off.numel() - 1
    _lengths(offsets=(n_cells + 1, a_off, b_off, pair_off), counts=(n_cells, a_cnt, b_cnt),
             cell_id=(n_cells, cell_id))
    n_pairs = int(pair_off[-1].item())
    dev = a_off.device
    pa = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    pb = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    nab = torch.empty(max(n_cells, 1), dtype=torch.float64, device=dev)
    _check(get_lib().cmc_pair_cells(n_cells, _ptr(cell_id, "int64"), _ptr(a_off, "int64"), _ptr(a_cnt, "int32"),
                              _ptr(b_off, "int64"),
                              _ptr(b_cnt, "int32"), _ptr(wa, "float64"), _ptr(wb, "float64"), int(seed),
                              int(step), int(pass_), _ptr(pair_off, "int64"),
                              _ptr(pa), _ptr(pb), _ptr(nab), _stream(stream)), "cmc_pair_cells")
    return pa[:n_pairs], pb[:n_pairs], nab[:n_cells]


def _species(d: Dict) -> _Species:
    s = _Species()
    s.off = _ptr(d["off"], "int64")
    s.count = _ptr(d.get("count"), "int32")
    for k in ("px", "py", "pz", "w"):
        setattr(s, k, _ptr(d.get(k), "float64"))
    s.parent = _ptr(d.get("parent"), "int64")
    return s


class StepState:
    """Per-step argument block: keeps ctypes structs (and tally tensors)
    alive so that repeated steps only update the step counter."""

    def __init__(self, tables: Tables, cells, electrons, photons, ions, new_el, new_po, *, dt,
                 seed=1, processes=BREMS | BH | TRIDENT, precision=FP64, schedule=SCHED_AUTO,
                 max_per_cell=None, near_rel=1e-6):
        import torch
        self.tables = tables
        n = cells["Zstar"].numel()
        dev = cells["Zstar"].device
        _lengths(cells=(n, cells["n_i"], cells["T_e"], cells.get("cell_id")))
        # every array must cover its species' offsets (read once, here)
        for name, d in zip(("electrons", "photons", "ions", "new_el", "new_po"),
                           (electrons, photons, ions, new_el, new_po)):
            _lengths(**{f"{name} off": (n + 1, d["off"]), f"{name} count": (n, d.get("count"))})
            end = int(d["off"][-1].item()) if d["off"].numel() else 0
            for k in ("px", "py", "pz", "w", "parent"):
                a = d.get(k)
                if a is not None and a.numel() < end:
                    raise ValueError(f"{name} {k}: {a.numel()} elements for offsets up to {end}")
        self.cells = _Cells(n, _ptr(cells["Zstar"], "float64"), _ptr(cells["n_i"], "float64"),
                            _ptr(cells["T_e"], "float64"), _ptr(cells.get("cell_id"), "int64"))
        self.sp = [_species(x) for x in (electrons, photons, ions, new_el, new_po)]
        if max_per_cell is None:
            def mx(d):
                o = d["off"]
                return int((o[1:] - o[:-1]).max().item()) if o.numel() > 1 else 0
            max_per_cell = max(1, mx(electrons), mx(photons), mx(ions))
        self.params = _StepParams(float(dt), int(seed), 0, int(processes), int(precision),
                                  int(schedule), int(max_per_cell), float(near_rel))
        self.ti = torch.zeros((n, len(I_NAMES)), dtype=torch.int64, device=dev)
        self.td = torch.zeros((n, len(D_NAMES)), dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.tal = _Tallies(_ptr(self.ti), _ptr(self.td), _ptr(self.status))
        wsb = get_lib().cmc_step_workspace_bytes(n, int(schedule))
        self.workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev) if wsb else None
        self.wsb = wsb
        self._refs = (cells, electrons, photons, ions, new_el, new_po)
        self.counter = None

    def set_tallies(self, ti=None, td=None):
        """Write the next steps' integer (ti, int64 [n_cells, 12]) and FP64
        (td, [n_cells, 10]) tallies to other device tensors (None: the
        state's own), e.g. one row block per step."""
        for t, own, dt_ in ((ti, self.ti, "int64"), (td, self.td, "float64")):
            if t is not None and (tuple(t.shape) != tuple(own.shape)):
                raise ValueError(f"tallies: expected shape {tuple(own.shape)}, got {tuple(t.shape)}")
        self.tal.ti = _ptr(ti if ti is not None else self.ti, "int64")
        self.tal.td = _ptr(td if td is not None else self.td, "float64")
        self._tal_refs = (ti, td)

    def use_counter(self, counter):
        """Read the step number from `counter` (a one-element int64 device
        tensor) on the device; every step then advances it (None: back to
        the host step number)."""
        self.counter = counter
        self.params.step_counter = _ptr(counter) if counter is not None else None

    def graph(self, step0: int):
        """Capture one step in a HIP graph (torch.cuda.CUDAGraph) whose
        replays run steps step0, step0 + 1, ... (the step number lives in
        device memory).  Run the launch shape eagerly once before, so that
        the team shape is already tuned.  Returns (graph, counter)."""
        import torch
        counter = torch.tensor([int(step0)], dtype=torch.int64, device=self.ti.device)
        self.use_counter(counter)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            self.step(0)
        torch.cuda.current_stream().wait_stream(side)
        return g, counter

    def step(self, step: int, stream=None, events=None, noalloc=False):
        """One step; `events` = optional pair of raw hipEvent_t handles
        recorded around the pair-test kernels.  noalloc: through
        cmc_collide_step_noalloc (the library's static workspace) instead of
        this state's workspace."""
        self.params.step = int(step)
        self.params.pass_events[0] = events[0] if events else None
        self.params.pass_events[1] = events[1] if events else None
        if noalloc:
            _check(get_lib().cmc_collide_step_noalloc(self.tables.handle, C.byref(self.cells), C.byref(self.sp[0]),
                                                      C.byref(self.sp[1]), C.byref(self.sp[2]), C.byref(self.sp[3]),
                                                      C.byref(self.sp[4]), C.byref(self.params), C.byref(self.tal),
                                                      _stream(stream)),
                   "cmc_collide_step_noalloc")
            return
        _check(get_lib().cmc_collide_step(self.tables.handle, C.byref(self.cells), C.byref(self.sp[0]),
                                    C.byref(self.sp[1]), C.byref(self.sp[2]), C.byref(self.sp[3]),
                                    C.byref(self.sp[4]), C.byref(self.params), C.byref(self.tal),
                                    _ptr(self.workspace), self.wsb, _stream(stream)),
               "cmc_collide_step")


def collide_step(tables: Tables, cells, electrons, photons, ions, new_el, new_po, *, dt, seed, step,
                 processes=BREMS | BH | TRIDENT, precision=FP64, schedule=SCHED_AUTO,
                 max_per_cell=None, near_rel=1e-6, stream=None):
    """One Monte Carlo step in place on the given device tensors (dicts of
    torch tensors laid out as in include/cmc.h); returns (ti, td, status)
    tensors of per-cell tallies."""
    st = StepState(tables, cells, electrons, photons, ions, new_el, new_po, dt=dt, seed=seed,
                   processes=processes, precision=precision, schedule=schedule,
                   max_per_cell=max_per_cell, near_rel=near_rel)
    st.step(step, stream)
    return st.ti, st.td, st.status


_OFF_OK = {}


def _check_offsets(off, n_part):
    """off must start at 0, never decrease and end at or below n_part.  The
    check reads off from the device once per (tensor, version): repeated
    calls on the same offsets do not wait for the device.  The kernels
    check every cell again on the device (CMC_ST_BAD_OFFSETS)."""
    import weakref
    key = (id(off), off._version, int(n_part))
    ref = _OFF_OK.get(key)
    if ref is not None and ref() is off:
        return
    o = off.detach().cpu().numpy()
    if o.size == 0 or o[0] != 0 or np.any(np.diff(o) < 0) or o[-1] > n_part:
        raise ValueError("off must start at 0, be non-decreasing and end at or below the number of electrons "
                         f"({n_part})")
    if len(_OFF_OK) > 64:
        _OFF_OK.clear()
    _OFF_OK[key] = weakref.ref(off)


def expected_yield(tables: Tables, Zstar, n_e, T_e, off, px, py, pz, w, dt, precision=FP64,
                   per_particle=False, stream=None, status=None):
    """Y[c] = sum_j w_j P_j <k>_j per cell (cmc_expected_yield).  status: an
    optional int32 device tensor [1] OR-ed with CMC_ST_* bits (bad cells are
    skipped with Y = 0)."""
    import torch
    n = Zstar.numel()
    _lengths(cells=(n, n_e, T_e), off=(n + 1, off), electrons=(px.numel(), py, pz, w), status=(1, status))
    _check_offsets(off, px.numel())
    Y = torch.empty(n, dtype=torch.float64, device=Zstar.device)
    yp = torch.empty_like(px) if per_particle else None
    f8 = "float64"
    _check(get_lib().cmc_expected_yield(tables.handle, n, _ptr(Zstar, f8), _ptr(n_e, f8), _ptr(T_e, f8),
                                  _ptr(off, "int64"), px.numel(), _ptr(px, f8), _ptr(py, f8), _ptr(pz, f8),
                                  _ptr(w, f8), float(dt), int(precision),
                                  _ptr(Y), _ptr(yp), _ptr(status, "int32"), _stream(stream)),
           "cmc_expected_yield")
    return (Y, yp) if per_particle else Y


def expected_yield_backward(tables: Tables, Zstar, n_e, T_e, off, px, py, pz, w, dt, gY,
                            precision=FP64, stream=None, status=None, weight_grad=True):
    """The adjoint of expected_yield (cmc_expected_yield_backward): a dict of
    gpx, gpy, gpz, gZstar, gn_e, gT_e and, with weight_grad, gw."""
    import torch
    n = Zstar.numel()
    _lengths(cells=(n, n_e, T_e, gY), off=(n + 1, off), electrons=(px.numel(), py, pz, w), status=(1, status))
    _check_offsets(off, px.numel())
    out = {k: torch.empty_like(px) for k in (("gpx", "gpy", "gpz", "gw") if weight_grad else ("gpx", "gpy", "gpz"))}
    out.update({k: torch.empty_like(Zstar) for k in ("gZstar", "gn_e", "gT_e")})
    f8 = "float64"
    _check(get_lib().cmc_expected_yield_backward(
        tables.handle, Zstar.numel(), _ptr(Zstar, f8), _ptr(n_e, f8), _ptr(T_e, f8), _ptr(off, "int64"),
        px.numel(), _ptr(px, f8), _ptr(py, f8), _ptr(pz, f8), _ptr(w, f8), float(dt), int(precision),
        _ptr(gY.contiguous(), f8),
        _ptr(out["gpx"]), _ptr(out["gpy"]), _ptr(out["gpz"]), _ptr(out.get("gw")), _ptr(out["gZstar"]),
        _ptr(out["gn_e"]), _ptr(out["gT_e"]), _ptr(status, "int32"), _stream(stream)),
        "cmc_expected_yield_backward")
    return out


def merge_species(dst: Dict, src: Dict, stream=None, status=None, dropped=False):
    """Append src's live particles to dst's, cell by cell, as far as dst's
    slabs hold them; src is emptied (cmc_merge_species).  Both need
    'count'.  dropped=True: also return the dropped count per cell."""
    import torch
    n = dst["off"].numel() - 1
    _lengths(cells=(n, dst.get("count"), src.get("count")), offsets=(n + 1, src["off"]), status=(1, status))
    dr = torch.empty(n, dtype=torch.int64, device=dst["off"].device) if dropped else None
    d, s = _species(dst), _species(src)
    _check(get_lib().cmc_merge_species(n, C.byref(d), C.byref(s), _ptr(dr), _ptr(status, "int32"),
                                       _stream(stream)), "cmc_merge_species")
    return dr


def rebin(sp: Dict, headroom: int, stream=None) -> Dict:
    """A copy of species sp in new slabs on the device: each cell's live
    particles, then headroom free slots (cmc_rebin_offsets, then
    cmc_rebin_copy; the new total is read on the host in between)."""
    import torch
    n = sp["off"].numel() - 1
    dev = sp["off"].device
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    src = _species(sp)
    _check(get_lib().cmc_rebin_offsets(n, C.byref(src), int(headroom), _ptr(off), _stream(stream)),
           "cmc_rebin_offsets")
    m = int(off[-1].item())
    out = {"off": off, "count": torch.zeros(n, dtype=torch.int32, device=dev)}
    for k in ("px", "py", "pz", "w"):
        out[k] = torch.zeros(m, dtype=torch.float64, device=dev) if sp.get(k) is not None else None
    out["parent"] = (torch.full((m,), -1, dtype=torch.int64, device=dev) if sp.get("parent") is not None
                     else None)
    dst = _species(out)
    _check(get_lib().cmc_rebin_copy(n, C.byref(src), C.byref(dst), _stream(stream)), "cmc_rebin_copy")
    return out


def screening_functions(tables: Tables, Zstar, n_i, T_e, delta, form=SCREEN_REDUCED, stream=None, status=None):
    """(I1, I2) at delta per point, each with its cell state, in the reduced
    or the two-exponential form (cmc_screening_functions).  status: an
    optional int32 device tensor [1] OR-ed with CMC_ST_* bits."""
    import torch
    n = Zstar.numel()
    _lengths(points=(n, n_i, T_e, delta), status=(1, status))
    I1 = torch.empty(n, dtype=torch.float64, device=Zstar.device)
    I2 = torch.empty_like(I1)
    f8 = "float64"
    _check(get_lib().cmc_screening_functions(tables.handle, int(form), n, _ptr(Zstar, f8), _ptr(n_i, f8),
                                             _ptr(T_e, f8), _ptr(delta, f8), _ptr(I1), _ptr(I2),
                                             _ptr(status, "int32"), _stream(stream)),
           "cmc_screening_functions")
    return I1, I2


def cross_sections(tables: Tables, process, Zstar, n_i, T_e, e1, x, form=SCREEN_REDUCED, stream=None,
                   status=None):
    """k dsigma/dk (process BREMS: e1 = gamma_1, x = k/(gamma_1 - 1)) or
    dsigma/dgamma_+ (process BH: e1 = k, x = (gamma_+ - 1)/(k - 2)) per
    point, in m^2, in the reduced or the two-exponential screening form
    (cmc_cross_sections)."""
    import torch
    n = Zstar.numel()
    _lengths(points=(n, n_i, T_e, e1, x), status=(1, status))
    out = torch.empty(n, dtype=torch.float64, device=Zstar.device)
    f8 = "float64"
    _check(get_lib().cmc_cross_sections(tables.handle, int(process), int(form), n, _ptr(Zstar, f8), _ptr(n_i, f8),
                                        _ptr(T_e, f8), _ptr(e1, f8), _ptr(x, f8), _ptr(out),
                                        _ptr(status, "int32"), _stream(stream)),
           "cmc_cross_sections")
    return out


def _autograd_function():
    import torch

    class ExpectedYield(torch.autograd.Function):
        """Y[c] = sum_j w_j P_j <k>_j per cell; differentiable in px, py, pz, w,
        Z*, n_e and T_e through the hand-written adjoint kernel (the table
        lookups are recomputed in backward; only the inputs are saved)."""

        @staticmethod
        def forward(ctx, px, py, pz, w, Zstar, n_e, T_e, off, tables, dt, precision=FP64):
            ctx.save_for_backward(px, py, pz, w, Zstar, n_e, T_e, off)
            ctx.tables, ctx.dt, ctx.precision = tables, dt, precision
            return expected_yield(tables, Zstar, n_e, T_e, off, px, py, pz, w, dt, precision)

        @staticmethod
        def backward(ctx, gY):
            px, py, pz, w, Zstar, n_e, T_e, off = ctx.saved_tensors
            g = expected_yield_backward(ctx.tables, Zstar, n_e, T_e, off, px, py, pz, w, ctx.dt,
                                        gY.to(torch.float64), ctx.precision, weight_grad=ctx.needs_input_grad[3])
            return (g["gpx"], g["gpy"], g["gpz"], g.get("gw"), g["gZstar"], g["gn_e"], g["gT_e"],
                    None, None, None, None)

    return ExpectedYield


try:
    ExpectedYield = _autograd_function()
except Exception:  # torch missing: the C ABI stays usable without autograd
    ExpectedYield = None
