"""ctypes wrapper of the FP64 CPU oracle (oracle/cmc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check of
__graft_entry__ and by the CPU-baseline leg of bench.py, never by the
product package.  Arrays are numpy (host memory); species are dicts with the
keys ``off`` (int64 [n_cells+1]), ``count`` (int32 [n_cells] or None),
``px``, ``py``, ``pz``, ``w`` (float64) and ``parent`` (int64 or None).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

BREMS, BH, TRIDENT = 1, 2, 4

# tallies, same order as cmc_oracle.h
I_NAMES = ["pairs_br", "pairs_tr", "pairs_bh", "ev_br", "ev_tr", "ev_bh",
           "near_br", "near_tr", "near_bh", "drop_ph", "drop_el", "drop_po"]
D_NAMES = ["nab_ei", "nab_gi", "E_br", "E_tr", "E_bh", "dE_el", "dE_ph",
           "W_br", "W_tr", "W_bh"]
ST_OVERFLOW, ST_GAMMA_HIGH, ST_BAD_CELL, ST_BAD_WEIGHT = 1, 2, 4, 8

TABLE_NAMES = ["sigR", "skR", "cdfR", "sigU", "skU", "cdfU", "sigN", "skN", "cdfN",
               "sigB", "cdfB", "cdfT", "cdfS"]

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_u32p = C.POINTER(C.c_uint32)


class _Cells(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("Zstar", _dp), ("n_i", _dp), ("T_e", _dp),
                ("cell_id", _i64p)]


class _Species(C.Structure):
    _fields_ = [("off", _i64p), ("count", _i32p), ("px", _dp), ("py", _dp), ("pz", _dp),
                ("w", _dp), ("parent", _i64p)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle import build as _b  # noqa: F401  (build on first use)
            _b.build()
        L = C.CDLL(path)
        d, i32, i64, u64, u32 = C.c_double, C.c_int32, C.c_int64, C.c_uint64, C.c_uint32
        vp = C.c_void_p
        L.or_tables_build.argtypes = [C.c_int, C.POINTER(vp)]
        L.or_tables_free.argtypes = [vp]
        L.or_tables_size.argtypes = [vp, C.c_int]
        L.or_tables_size.restype = i64
        L.or_tables_export.argtypes = [vp, C.c_int, _dp, i64]
        L.or_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
        L.or_lambert_w0.argtypes = [d]; L.or_lambert_w0.restype = d
        L.or_fc.argtypes = [d]; L.or_fc.restype = d
        L.or_I12.argtypes = [d, d, _dp, _dp]
        L.or_I_tfd.argtypes = [d, d, d, d]; L.or_I_tfd.restype = d
        L.or_I12_tfd.argtypes = [d, d, d, d, d, _dp, _dp]
        L.or_dsdk_rel_tfd.argtypes = [d, d, d, d, d, d, d, C.c_int]; L.or_dsdk_rel_tfd.restype = d
        L.or_dsdgp_bh_tfd.argtypes = [d, d, d, d, d, d, d]; L.or_dsdgp_bh_tfd.restype = d
        L.or_L_reduced.argtypes = [d]; L.or_L_reduced.restype = d
        L.or_screening.argtypes = [d, d, d, d, _dp]
        L.or_dsdk_nr.argtypes = [d, d, d, d, d, d, C.c_int]; L.or_dsdk_nr.restype = d
        L.or_dsdk_rel.argtypes = [d, d, d, d, C.c_int]; L.or_dsdk_rel.restype = d
        L.or_dsdgp_bh.argtypes = [d, d, d, d]; L.or_dsdgp_bh.restype = d
        L.or_sigma_trident.argtypes = [d, d]; L.or_sigma_trident.restype = d
        L.or_dsdgp_trident.argtypes = [d, d, d]; L.or_dsdgp_trident.restype = d
        L.or_split_shape.argtypes = [d, d]; L.or_split_shape.restype = d
        L.or_philox.argtypes = [_u32p, _u32p, _u32p]
        L.or_u53.argtypes = [u32, u32]; L.or_u53.restype = d
        L.or_accept_uniforms.argtypes = [u64, u64, u32, u32, u32, u32, _dp, _dp]
        L.or_merge_species.argtypes = [i64, C.POINTER(_Species), C.POINTER(_Species), _i64p]
        L.or_rebin_offsets.argtypes = [i64, C.POINTER(_Species), C.c_int32, _i64p]
        L.or_rebin_copy.argtypes = [i64, C.POINTER(_Species), C.POINTER(_Species)]
        L.or_to_ion.argtypes = [_dp, d, _dp, _dp]
        L.or_from_ion.argtypes = [_dp, d, _dp, _dp]
        L.or_lookup.argtypes = [vp, d, d, d, d, C.c_int, _dp]
        L.or_sample.argtypes = [vp, d, d, d, d, C.c_int, d, d, _dp]
        L.or_pair_cells.argtypes = [i64, _i64p, _i64p, _i32p, _i64p, _i32p, _dp, _dp, u64, u64, u32,
                                    _i64p, _i32p, _i32p, _dp]
        L.or_collide_step.argtypes = [vp, C.POINTER(_Cells), C.POINTER(_Species),
                                      C.POINTER(_Species), C.POINTER(_Species),
                                      C.POINTER(_Species), C.POINTER(_Species),
                                      d, u64, u64, u32, d, _i64p, _dp, _i32p, C.c_int]
        L.or_expected_yield.argtypes = [vp, i64, _dp, _dp, _dp, _i64p, _dp, _dp, _dp, _dp, d,
                                        _dp, _dp, C.c_int]
        L.or_expected_yield_backward.argtypes = [vp, i64, _dp, _dp, _dp, _i64p, _dp, _dp, _dp,
                                                 _dp, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                                 _dp, _dp, C.c_int]
        _LIB = L
    return _LIB


def _p(a, ct=_dp):
    if a is None:
        return ct()
    assert a.flags["C_CONTIGUOUS"], "arrays must be contiguous"
    return a.ctypes.data_as(ct)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- physics
def gauss_legendre(n):
    x = np.zeros(n); w = np.zeros(n)
    lib().or_gauss_legendre(n, _p(x), _p(w))
    return x, w


def lambert_w0(z):
    return lib().or_lambert_w0(float(z))


def fc(Z):
    return lib().or_fc(float(Z))


def I12(delta, L):
    a = C.c_double(); b = C.c_double()
    lib().or_I12(float(delta), float(L), C.byref(a), C.byref(b))
    return a.value, b.value


def I_tfd(etf, ed, Ltf, Ld):
    return lib().or_I_tfd(float(etf), float(ed), float(Ltf), float(Ld))


def I12_tfd(delta, etf, ed, Ltf, Ld):
    """eq:defphi1, eq:defphi2 for the two-exponential potential eq:V_TFD
    (quadrature of the definitions)."""
    a = C.c_double(); b = C.c_double()
    lib().or_I12_tfd(float(delta), float(etf), float(ed), float(Ltf), float(Ld), C.byref(a), C.byref(b))
    return a.value, b.value


def dsdk_rel_tfd(Z, g1, k, etf, ed, Ltf, Ld, coulomb=False):
    return lib().or_dsdk_rel_tfd(float(Z), float(g1), float(k), float(etf), float(ed), float(Ltf), float(Ld),
                                 int(coulomb))


def dsdgp_bh_tfd(Z, k, gp, etf, ed, Ltf, Ld):
    return lib().or_dsdgp_bh_tfd(float(Z), float(k), float(gp), float(etf), float(ed), float(Ltf), float(Ld))


def L_reduced(a):
    return lib().or_L_reduced(float(a))


def screening(Z, Zs, ni, T):
    """-> dict(Ltf, Ld, etf, ed, a, Lr, branch, ri)"""
    out = np.zeros(8)
    lib().or_screening(float(Z), float(Zs), float(ni), float(T), _p(out))
    keys = ["Ltf", "Ld", "etf", "ed", "a", "Lr", "branch", "ri"]
    return dict(zip(keys, out.tolist()))


def dsdk_nr(Z, g1, k, eta_d, Ltf, Ld, elwert=True):
    return lib().or_dsdk_nr(float(Z), float(g1), float(k), float(eta_d), float(Ltf), float(Ld),
                            int(elwert))


def dsdk_rel(Z, g1, k, L, coulomb=False):
    return lib().or_dsdk_rel(float(Z), float(g1), float(k), float(L), int(coulomb))


def dsdgp_bh(Z, k, gp, L):
    return lib().or_dsdgp_bh(float(Z), float(k), float(gp), float(L))


def sigma_trident(Z, g1):
    return lib().or_sigma_trident(float(Z), float(g1))


def dsdgp_trident(Z, g1, gpair):
    return lib().or_dsdgp_trident(float(Z), float(g1), float(gpair))


def split_shape(gpair, gplus):
    return lib().or_split_shape(float(gpair), float(gplus))


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox(_p(c, _u32p), _p(k, _u32p), _p(o, _u32p))
    return o


def to_ion(u, E, p):
    """(E', p') of the 4-vector (E, p) in the rest frame of an ion of
    proper velocity u (Sec. III.A)."""
    out = np.zeros(4)
    lib().or_to_ion(_p(_f64(u)), float(E), _p(_f64(p)), _p(out))
    return out[0], out[1:]


def from_ion(u, Ep, pp):
    """Lab momentum of the ion-frame 4-vector (E', p')."""
    out = np.zeros(3)
    lib().or_from_ion(_p(_f64(u)), float(Ep), _p(_f64(pp)), _p(out))
    return out


def u53(a, b):
    return lib().or_u53(int(a), int(b))


# tags of the acceptance draws: (pair's own draw, shared draw of U1's upper bits)
ACC_TAGS = {"br": (0x11, 0x13), "tr": (0x21, 0x23), "bh": (0x31, 0x33)}


def accept_uniforms(seed, step, cell, x, proc="bh"):
    """(U1, U2) of the acceptance test of the pair keyed by x."""
    u1, u2 = C.c_double(), C.c_double()
    tag, tag_hi = ACC_TAGS[proc]
    lib().or_accept_uniforms(int(seed), int(step), int(cell), int(x), tag, tag_hi, C.byref(u1), C.byref(u2))
    return u1.value, u2.value


# ---------------------------------------------------------------- tables
class Tables:
    """Oracle tables for one element Z (built on construction)."""

    def __init__(self, Z):
        self.Z = int(Z)
        h = C.c_void_p()
        rc = lib().or_tables_build(self.Z, C.byref(h))
        if rc != 0:
            raise ValueError(f"or_tables_build({Z}) failed: {rc}")
        self._h = h

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().or_tables_free(self._h)
                self._h = None
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def export(self, name):
        which = TABLE_NAMES.index(name) if isinstance(name, str) else int(name)
        n = lib().or_tables_size(self._h, which)
        out = np.zeros(n)
        rc = lib().or_tables_export(self._h, which, _p(out), n)
        assert rc == 0
        return out

    def lookup(self, Zs, ni, T, e1, process):
        out = np.zeros(4)
        lib().or_lookup(self._h, float(Zs), float(ni), float(T), float(e1), int(process), _p(out))
        return out

    def sample(self, Zs, ni, T, e1, process, xi1, xi2=0.5):
        out = np.zeros(2)
        rc = lib().or_sample(self._h, float(Zs), float(ni), float(T), float(e1), int(process),
                             float(xi1), float(xi2), _p(out))
        return None if rc else out


_TABLE_CACHE = {}


def tables(Z):
    """Cached oracle tables for element Z."""
    if Z not in _TABLE_CACHE:
        _TABLE_CACHE[Z] = Tables(Z)
    return _TABLE_CACHE[Z]


# ---------------------------------------------------------------- step
def pair_cells(a_off, a_cnt, b_off, b_cnt, wa, wb, seed, step, pass_, pair_off, cell_id=None):
    """Pair indices of every cell; cell_id (int64, or None = position) is the
    global cell index that keys the draws."""
    n_cells = len(a_off) - 1
    cid = None if cell_id is None else np.ascontiguousarray(cell_id, np.int64)
    n_pairs = int(pair_off[-1])
    pa = np.zeros(max(n_pairs, 1), dtype=np.int32)
    pb = np.zeros(max(n_pairs, 1), dtype=np.int32)
    nab = np.zeros(n_cells)
    a_off = np.ascontiguousarray(a_off, np.int64); b_off = np.ascontiguousarray(b_off, np.int64)
    a_cnt = None if a_cnt is None else np.ascontiguousarray(a_cnt, np.int32)
    b_cnt = None if b_cnt is None else np.ascontiguousarray(b_cnt, np.int32)
    pair_off = np.ascontiguousarray(pair_off, np.int64)
    rc = lib().or_pair_cells(n_cells, _p(cid, _i64p), _p(a_off, _i64p), _p(a_cnt, _i32p), _p(b_off, _i64p),
                             _p(b_cnt, _i32p), _p(_f64(wa)), _p(_f64(wb)), int(seed), int(step),
                             int(pass_), _p(pair_off, _i64p), _p(pa, _i32p), _p(pb, _i32p),
                             _p(nab))
    assert rc == 0
    return pa[:n_pairs], pb[:n_pairs], nab


def _species(d):
    s = _Species()
    s.off = _p(d["off"], _i64p)
    s.count = _p(d.get("count"), _i32p)
    for k in ("px", "py", "pz", "w"):
        setattr(s, k, _p(d.get(k)))
    s.parent = _p(d.get("parent"), _i64p)
    return s


def collide_step(tab, cells, electrons, photons, ions, new_el, new_po, dt, seed, step,
                 processes=BREMS | BH | TRIDENT, near_rel=1e-6, nthreads=0):
    """Runs one step in place on the dict arrays; returns (tal_i, tal_d, status)."""
    n = len(cells["Zstar"])
    keep = [_f64(cells["Zstar"]), _f64(cells["n_i"]), _f64(cells["T_e"])]
    cid = cells.get("cell_id")
    cid = None if cid is None else np.ascontiguousarray(cid, np.int64)
    cs = _Cells(n, _p(keep[0]), _p(keep[1]), _p(keep[2]), _p(cid, _i64p))
    sp = [_species(x) for x in (electrons, photons, ions, new_el, new_po)]
    ti = np.zeros((n, len(I_NAMES)), dtype=np.int64)
    td = np.zeros((n, len(D_NAMES)))
    st = np.zeros(1, dtype=np.int32)
    rc = lib().or_collide_step(tab.handle, C.byref(cs), C.byref(sp[0]), C.byref(sp[1]),
                               C.byref(sp[2]), C.byref(sp[3]), C.byref(sp[4]), float(dt),
                               int(seed), int(step), int(processes), float(near_rel),
                               _p(ti, _i64p), _p(td), _p(st, _i32p), int(nthreads))
    if rc != 0:
        raise ValueError(f"or_collide_step failed: {rc}")
    return ti, td, int(st[0])


def expected_yield(tab, Zs, n_e, T_e, off, px, py, pz, w, dt, per_particle=False, nthreads=0):
    n = len(Zs)
    Y = np.zeros(n)
    yp = np.zeros(len(px)) if per_particle else None
    arrs = [_f64(a) for a in (Zs, n_e, T_e)]
    pa = [_f64(a) for a in (px, py, pz, w)]
    off = np.ascontiguousarray(off, np.int64)
    lib().or_expected_yield(tab.handle, n, _p(arrs[0]), _p(arrs[1]), _p(arrs[2]),
                            _p(off, _i64p), _p(pa[0]), _p(pa[1]), _p(pa[2]), _p(pa[3]),
                            float(dt), _p(Y), _p(yp), int(nthreads))
    return (Y, yp) if per_particle else Y


def expected_yield_backward(tab, Zs, n_e, T_e, off, px, py, pz, w, dt, gY, nthreads=0, scale=False):
    """Adjoint of expected_yield; with scale=True also 'gabs': per cell and
    cell gradient (Z*, n_e, T_e), the sum of the magnitudes of the terms it
    is summed from (the scale of its rounding error in any summation order)."""
    n = len(Zs); m = len(px)
    arrs = [_f64(a) for a in (Zs, n_e, T_e, gY)]
    pa = [_f64(a) for a in (px, py, pz, w)]
    off = np.ascontiguousarray(off, np.int64)
    out = [np.zeros(m) for _ in range(4)] + [np.zeros(n) for _ in range(3)]
    gabs = np.zeros((n, 3)) if scale else None
    lib().or_expected_yield_backward(tab.handle, n, _p(arrs[0]), _p(arrs[1]), _p(arrs[2]),
                                     _p(off, _i64p), _p(pa[0]), _p(pa[1]), _p(pa[2]), _p(pa[3]),
                                     float(dt), _p(arrs[3]), *[_p(o) for o in out], _p(gabs),
                                     int(nthreads))
    keys = ["gpx", "gpy", "gpz", "gw", "gZstar", "gn_e", "gT_e"]
    res = dict(zip(keys, out))
    if scale:
        res["gabs"] = gabs
    return res


def merge_species(dst, src):
    """Append src's live particles to dst's, cell by cell, as far as dst's
    slabs hold them; src is emptied (the arrays are updated in place).
    dst and src need live counts.  Returns the dropped count per cell."""
    n = len(dst["off"]) - 1
    assert dst.get("count") is not None and src.get("count") is not None
    dropped = np.zeros(n, dtype=np.int64)
    d, s_ = _species(dst), _species(src)
    lib().or_merge_species(n, C.byref(d), C.byref(s_), _p(dropped, _i64p))
    return dropped


def rebin(sp, headroom):
    """A copy of species sp in new slabs: each cell's live particles, then
    headroom free slots (zeros)."""
    n = len(sp["off"]) - 1
    off = np.zeros(n + 1, dtype=np.int64)
    src = _species(sp)
    lib().or_rebin_offsets(n, C.byref(src), int(headroom), _p(off, _i64p))
    m = int(off[-1])
    out = {"off": off, "count": np.zeros(n, dtype=np.int32)}
    for k in ("px", "py", "pz", "w"):
        out[k] = np.zeros(m) if sp.get(k) is not None else None
    out["parent"] = np.full(m, -1, dtype=np.int64) if sp.get("parent") is not None else None
    dst = _species(out)
    lib().or_rebin_copy(n, C.byref(src), C.byref(dst))
    return out

