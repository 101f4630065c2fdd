"""Random numbers keyed by the global cell index (cmc_cells.cell_id, the
cell word of every Philox counter, Sec. III.A's per-cell pairing): the
cells of a workload split over two launches give the same results as one
launch over all of them, bit for bit; a subset launched with its global
indices matches the oracle run on the same subset."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_02814_amd import workloads as W

pytestmark = pytest.mark.gpu


def _wl():
    # uneven cells, all three processes, a time step amplified 200 times so
    # that every step has events in most cells (and sequential-step cells)
    return W.cfg3(np.random.default_rng(77), n_cells=96, lo=16, hi=600, dt=2e-14)


def _live(d, c):
    off = d["off"]
    n = int(d["count"][c]) if d.get("count") is not None else int(off[c + 1] - off[c])
    a = int(off[c])
    return [d[k][a:a + n] for k in ("px", "py", "pz", "w")] + ([d["parent"][a:a + n]] if d.get("parent") is not None else [])


def _host(g):
    return {k: (None if v is None else v.cpu().numpy()) for k, v in g.items()}


def test_two_half_launches_equal_one_launch():
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    wl = _wl()
    n = wl.n_cells
    parts = [np.arange(0, n // 2), np.arange(n // 2, n)]
    full = wl.copy().to_torch("cuda:0")
    halves = [wl.subset(p).to_torch("cuda:0") for p in parts]
    assert all("cell_id" in h.cells for h in halves)

    def state(g):
        return cmc.StepState(gpu_tables(wl.Z), g.cells, g.electrons, g.photons, g.ions, g.new_el, g.new_po,
                             dt=wl.dt, seed=1, processes=wl.processes, precision=cmc.FP64)
    sf = state(full)
    sh = [state(h) for h in halves]
    events = 0
    for s in range(3):
        sf.step(s)
        for x in sh:
            x.step(s)
        torch.cuda.synchronize()
        ti = sf.ti.cpu().numpy()
        events += int(ti[:, 3:6].sum())
        for p, x in zip(parts, sh):
            assert np.array_equal(ti[p], x.ti.cpu().numpy()), s
            assert np.array_equal(sf.td.cpu().numpy()[p], x.td.cpu().numpy()), s
        assert int(sf.status.item()) == (int(sh[0].status.item()) | int(sh[1].status.item()))
    # parents are indices into the launch's own electron or photon arrays:
    # the half launch's are shifted by its offset of the parent's species
    Fe, Fg = wl.electrons["off"], full.photons["off"].cpu().numpy()
    for name in ("electrons", "photons", "new_el", "new_po"):
        F = _host(getattr(full, name))
        for p, h in zip(parts, halves):
            H = _host(getattr(h, name))
            He, Hg = h.electrons["off"].cpu().numpy(), h.photons["off"].cpu().numpy()
            for li, c in enumerate(p):
                fa, ha = _live(F, c), _live(H, li)
                for a, b in zip(fa[:4], ha[:4]):
                    assert np.array_equal(a, b), (name, c)
                if len(fa) > 4:
                    d = fa[4] - ha[4]
                    shifts = (Fe[c] - He[li], Fg[c] - Hg[li])
                    ok = ((fa[4] == -1) & (ha[4] == -1)) | (d == shifts[0]) | (d == shifts[1])
                    assert np.all(ok), (name, c)
    print(f"[cell_id] {events} events over 3 steps, identical in two half launches")
    assert events > 100


def test_subset_with_global_indices_matches_the_oracle():
    import paper_1907_02814_amd as cmc
    from gpu_parity import Parity
    wl = _wl()
    sample = np.sort(np.random.default_rng(3).choice(wl.n_cells, 24, replace=False))
    sub = wl.subset(sample)
    assert np.array_equal(sub.cells["cell_id"], sample)
    for prec in (cmc.FP64, cmc.FP32):
        P = Parity(sub, precision=prec)
        for s in range(3):
            P.step(s)
        print(f"[cell_id] subset, precision {prec}: {P.flips} flip(s); "
              + ", ".join(f"{k} {v:.1e}" for k, v in P.errors.items()))
        assert P.flips <= 2


def test_pair_cells_with_global_indices():
    import torch
    import paper_1907_02814_amd as cmc
    rng = np.random.default_rng(8)
    n = 12
    na = rng.integers(1, 300, n)
    nb = rng.integers(1, 300, n)
    a_off = np.concatenate([[0], np.cumsum(na)]).astype(np.int64)
    b_off = np.concatenate([[0], np.cumsum(nb)]).astype(np.int64)
    p_off = np.concatenate([[0], np.cumsum(np.maximum(na, nb))]).astype(np.int64)
    wa, wb = rng.lognormal(0, 1, int(na.sum())), rng.lognormal(0, 1, int(nb.sum()))
    cid = np.sort(rng.choice(100000, n, replace=False)).astype(np.int64)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    pa, pb, nab = cmc.pair_cells(t(a_off), None, t(b_off), None, t(wa), t(wb), 4, 2, 2, t(p_off), cell_id=t(cid))
    opa, opb, onab = O.pair_cells(a_off, None, b_off, None, wa, wb, 4, 2, 2, p_off, cell_id=cid)
    assert np.array_equal(pa.cpu().numpy(), opa) and np.array_equal(pb.cpu().numpy(), opb)
    np.testing.assert_allclose(nab.cpu().numpy(), onab, rtol=1e-12)
    # and they are not the pairs of the cells numbered by position
    opa0, _, _ = O.pair_cells(a_off, None, b_off, None, wa, wb, 4, 2, 2, p_off)
    assert not np.array_equal(opa0, opa)
