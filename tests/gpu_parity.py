"""Helpers of the GPU parity tests: run the same seeded workload through the
HIP library (via the C ABI) and through the oracle, compare cell by cell.

Rules: event counts, slots and parent indices bit-exact; floating-point
outputs within `rtol` (1e-12 for the FP64 form, 1e-5 for the FP32 form).
A cell may differ only if it holds a decision within the near-threshold
band |U - P| <= 1e-6 P (counted by both sides); such cells are counted,
reported and left out of later comparisons.
"""
import functools
import sys

import numpy as np

import paper_1907_02814_amd as cmc
from paper_1907_02814_amd import D_NAMES
from oracle import oracle as O


def torch_mod():
    import torch
    return torch


DEV = "cuda:0"


@functools.lru_cache(maxsize=None)
def gpu_tables(Z):
    return cmc.build_tables(Z)


def tally_scale(otd):
    """Scale of each FP64 tally of each cell for its relative error: the
    tally itself for n_ab, the event energies E_br, E_tr, E_bh and the
    weights, sums of terms of one sign.  The energy changes dE_el and
    dE_ph can mix signs (with moving ions a lab-frame change may be a
    gain), so they are judged against the cell's energy throughput, the
    sum of the magnitudes of its energy tallies (the oracle does not report
    their terms)."""
    sc = np.abs(otd).astype(np.float64)
    pooled = np.abs(otd[:, 2:5]).sum(1) + np.abs(otd[:, 5:7]).sum(1)
    for q in (5, 6):
        sc[:, q] = np.maximum(sc[:, q], pooled)
    return sc


def _vec_rel(ax, ay, az, bx, by, bz):
    """|a - b|/|b| per particle (0 where both vanish)."""
    da = np.sqrt((ax - bx) ** 2 + (ay - by) ** 2 + (az - bz) ** 2)
    mag = np.sqrt(bx * bx + by * by + bz * bz)
    return np.where(da == 0, 0.0, da / np.maximum(mag, 1e-300))


class Parity:
    def __init__(self, wl, *, precision=cmc.FP64, schedule=cmc.SCHED_AUTO, seed=1,
                 max_per_cell=None, rtol=None, nthreads=0):
        torch = torch_mod()
        self.wl = wl
        self.ref = wl.copy()
        self.g = wl.to_torch(DEV)
        self.rtol = rtol if rtol is not None else (1e-12 if precision == cmc.FP64 else 1e-5)
        self.seed = seed
        self.nthreads = nthreads
        self.state = cmc.StepState(gpu_tables(wl.Z), self.g.cells, self.g.electrons, self.g.photons,
                                   self.g.ions, self.g.new_el, self.g.new_po, dt=wl.dt, seed=seed,
                                   processes=wl.processes, precision=precision, schedule=schedule,
                                   max_per_cell=max_per_cell)
        self.diverged = np.zeros(wl.n_cells, dtype=bool)
        self.flips = 0
        self.report = []
        self.torch = torch
        self.errors = {}

    def step(self, s):
        torch = self.torch
        self.state.status.zero_()
        self.state.step(s)
        torch.cuda.synchronize()
        oti, otd, ost = O.collide_step(O.tables(self.wl.Z), self.ref.cells, self.ref.electrons,
                                       self.ref.photons, self.ref.ions, self.ref.new_el,
                                       self.ref.new_po, self.wl.dt, self.seed, s, self.wl.processes,
                                       nthreads=self.nthreads)
        ti = self.state.ti.cpu().numpy()
        td = self.state.td.cpu().numpy()
        st = int(self.state.status.item())
        return self.compare(ti, td, st, oti, otd, ost, s)

    def _cells_of(self, off, n):
        return np.repeat(np.arange(n), np.diff(off))

    def _note(self, key, err):
        if err.size:
            self.errors[key] = max(self.errors.get(key, 0.0), float(np.max(err)))

    def compare(self, ti, td, st, oti, otd, ost, s):
        g, r, rtol = self.g, self.ref, self.rtol
        n = self.wl.n_cells
        bad = np.zeros(n, dtype=bool)
        why = {}

        def flag(mask, name):
            nonlocal bad
            for c in np.flatnonzero(mask & ~bad):
                why.setdefault(int(c), name)
            bad |= mask

        flag(np.any(ti != oti, axis=1), "ti")
        keep = ~self.diverged
        # electrons: per-particle relative error of the momentum vector
        e = {k: g.electrons[k].cpu().numpy() for k in ("px", "py", "pz")}
        ecell = self._cells_of(r.electrons["off"], n)
        err = _vec_rel(e["px"], e["py"], e["pz"], r.electrons["px"], r.electrons["py"], r.electrons["pz"])
        self._note("electron p", err[keep[ecell]])
        flag(np.bincount(ecell[err > rtol], minlength=n) > 0, "electrons")
        # photon species and product buffers
        for name in ("photons", "new_el", "new_po"):
            G = getattr(g, name); Rr = getattr(r, name)
            cnt = G["count"].cpu().numpy()
            flag(cnt != Rr["count"], name + " count")
            off = Rr["off"]
            live = np.zeros(int(off[-1]), dtype=bool)
            for c in range(n):
                live[off[c]:off[c] + min(cnt[c], Rr["count"][c])] = True
            cells = self._cells_of(off, n)
            arr = {k: G[k].cpu().numpy() for k in ("px", "py", "pz", "w")}
            errv = _vec_rel(arr["px"], arr["py"], arr["pz"], Rr["px"], Rr["py"], Rr["pz"])
            errw = np.abs(arr["w"] - Rr["w"]) / np.maximum(np.abs(Rr["w"]), 1e-300)
            sel = live & keep[cells]
            self._note(name + " p", errv[sel]); self._note(name + " w", errw[sel])
            wrong = live & ((errv > rtol) | (errw > rtol))
            if G.get("parent") is not None and Rr.get("parent") is not None:
                wrong |= live & (G["parent"].cpu().numpy() != Rr["parent"])
            flag(np.bincount(cells[wrong], minlength=n) > 0, name)
        # FP64 tallies (scales: tally_scale)
        S = tally_scale(otd)
        for q in range(otd.shape[1]):
            ref = otd[:, q]
            sc = S[:, q]
            errq = np.abs(td[:, q] - ref) / np.maximum(sc, 1e-300)
            self._note("tally " + D_NAMES[q], errq[keep])
            flag(errq > rtol, "tally " + D_NAMES[q])
        new_bad = bad & ~self.diverged
        near = (oti[:, 6:9].sum(1) > 0) | (ti[:, 6:9].sum(1) > 0)
        unexplained = new_bad & ~near
        if unexplained.any():
            c = int(np.flatnonzero(unexplained)[0])
            msg = (f"step {s}: cell {c} differs ({why.get(c)}) without a near-threshold decision\n"
                   f"  errors so far {self.errors}\n"
                   f"  gpu ti {ti[c].tolist()}\n  ora ti {oti[c].tolist()}\n"
                   f"  gpu td {td[c].tolist()}\n  ora td {otd[c].tolist()}")
            raise AssertionError(msg)
        self.flips += int(new_bad.sum())
        self.diverged |= new_bad
        if new_bad.any():
            self.report.append((s, np.flatnonzero(new_bad).tolist()))
            print(f"[parity] step {s}: {int(new_bad.sum())} cell(s) with a near-threshold flip",
                  file=sys.stderr)
        assert (st & ~cmc.ST_OVERFLOW) == (ost & ~cmc.ST_OVERFLOW) or self.flips, (st, ost)
        return ti, td, oti, otd



def compare_sampled_cells(g, st, ref, sample, oti, otd, rtol):
    """GPU outputs (torch dict workload `g`, StepState `st`) of the cells
    `sample` against the oracle's (oti, otd, and the arrays of ref =
    wl.subset(sample), run from the same state: same global cell ids, hence
    the same random numbers).  Cells with a near-threshold decision on either
    side are left out; returns their number.  Raises on any other
    difference: integer tallies and counts bit-exact, floating point within
    rtol."""
    ti = st.ti.cpu().numpy()[sample]
    td = st.td.cpu().numpy()[sample]
    skip = (oti[:, 6:9].sum(1) > 0) | (ti[:, 6:9].sum(1) > 0)
    keep = ~skip
    if not np.array_equal(ti[keep], oti[keep]):
        c = int(np.flatnonzero(np.any(ti != oti, axis=1) & keep)[0])
        raise AssertionError(f"integer tallies of cell {sample[c]}: {ti[c].tolist()} vs {oti[c].tolist()}")
    err = np.abs(td - otd) / np.maximum(tally_scale(otd), 1e-300)
    if keep.any() and err[keep].max() > rtol:
        raise AssertionError(f"FP tallies differ by {err[keep].max():.3g}")
    for name in ("electrons", "photons", "new_el", "new_po"):
        G = getattr(g, name)
        Rr = getattr(ref, name)
        off_g = G["off"].cpu().numpy()
        arr = {k: G[k].cpu().numpy() for k in ("px", "py", "pz", "w")}
        cnt = G["count"].cpu().numpy() if G.get("count") is not None else np.diff(off_g)
        rcnt = Rr["count"] if Rr.get("count") is not None else np.diff(Rr["off"])
        for li, c in enumerate(sample):
            if skip[li]:
                continue
            n = int(cnt[c])
            if n != int(rcnt[li]):
                raise AssertionError(f"{name} count differs in cell {c}: {n} vs {rcnt[li]}")
            a0, r0 = int(off_g[c]), int(Rr["off"][li])
            ga = [arr[k][a0:a0 + n] for k in ("px", "py", "pz", "w")]
            ra = [Rr[k][r0:r0 + n] for k in ("px", "py", "pz", "w")]
            ev = _vec_rel(ga[0], ga[1], ga[2], ra[0], ra[1], ra[2])
            ew = np.abs(ga[3] - ra[3]) / np.maximum(np.abs(ra[3]), 1e-300)
            if n and (ev.max() > rtol or ew.max() > rtol):
                raise AssertionError(f"{name} of cell {c} differ: p {ev.max():.3g} w {ew.max():.3g}")
    return int(skip.sum())


def compare_host_subsets(ti, td, now, ref, oti, otd, rtol, skip_cells=None):
    """The GPU's state of some cells (`now`: Workload.host_subset of the
    device workload after the step; ti, td: their tally rows) against the
    oracle's state of the same cells (`ref`, stepped from the same state,
    same global cell ids; oti, otd its tallies).  Integer tallies and counts
    bit-exact, floating point within rtol.  Cells with a near-threshold
    decision on either side, and those in skip_cells (diverged earlier), are
    left out.  Returns the mask of cells left out and the largest errors."""
    n = len(ti)
    skip = (oti[:, 6:9].sum(1) > 0) | (ti[:, 6:9].sum(1) > 0)
    if skip_cells is not None:
        skip |= skip_cells
    keep = ~skip
    errs = {}
    bad = np.any(ti != oti, axis=1) & keep
    if bad.any():
        c = int(np.flatnonzero(bad)[0])
        raise AssertionError(f"integer tallies of cell {c}: {ti[c].tolist()} vs {oti[c].tolist()}")
    err = np.abs(td - otd) / np.maximum(tally_scale(otd), 1e-300)
    errs["tallies"] = float(err[keep].max()) if keep.any() else 0.0
    if errs["tallies"] > rtol:
        raise AssertionError(f"FP tallies differ by {errs['tallies']:.3g}")
    for name in ("electrons", "photons", "new_el", "new_po"):
        G, Rr = getattr(now, name), getattr(ref, name)
        gc = G["count"] if G.get("count") is not None else np.diff(G["off"])
        rc = Rr["count"] if Rr.get("count") is not None else np.diff(Rr["off"])
        worst = 0.0
        for c in np.flatnonzero(keep):
            if int(gc[c]) != int(rc[c]):
                raise AssertionError(f"{name} count differs in cell {c}: {gc[c]} vs {rc[c]}")
            m = int(gc[c])
            if m == 0:
                continue
            a0, r0 = int(G["off"][c]), int(Rr["off"][c])
            ga = [G[k][a0:a0 + m] for k in ("px", "py", "pz", "w")]
            ra = [Rr[k][r0:r0 + m] for k in ("px", "py", "pz", "w")]
            ev = _vec_rel(ga[0], ga[1], ga[2], ra[0], ra[1], ra[2])
            ew = np.abs(ga[3] - ra[3]) / np.maximum(np.abs(ra[3]), 1e-300)
            worst = max(worst, float(ev.max()), float(ew.max()))
            if ev.max() > rtol or ew.max() > rtol:
                raise AssertionError(f"{name} of cell {c} differ: p {ev.max():.3g} w {ew.max():.3g}")
        errs[name] = worst
    return skip, errs
