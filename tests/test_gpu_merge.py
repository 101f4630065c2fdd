"""The step after on the GPU (cmc_merge_species, cmc_rebin_offsets,
cmc_rebin_copy) against the oracle: bit-exact data movement on random
slabs, and chained steps in which the created electrons and positrons
join their populations between steps (Sec. III.A products, the chains of
Sec. IV), compared with the oracle step by step."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_02814_amd import workloads as W

pytestmark = pytest.mark.gpu


def _host_sp(rng, cap, cnt, parent=True):
    off = np.concatenate([[0], np.cumsum(cap)]).astype(np.int64)
    m = int(off[-1])
    return {"off": off, "count": np.asarray(cnt, dtype=np.int32), "px": rng.normal(size=m),
            "py": rng.normal(size=m), "pz": rng.normal(size=m), "w": rng.random(m),
            "parent": rng.integers(0, 1 << 40, m) if parent else None}


def _dev(d):
    import torch
    return {k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v)).cuda()) for k, v in d.items()}


def _eq(g, h, what):
    for k, v in h.items():
        if v is None:
            assert g.get(k) is None, (what, k)
            continue
        a = g[k].cpu().numpy()
        assert np.array_equal(a, v), (what, k, np.flatnonzero(a != v)[:5])


@pytest.mark.parametrize("n", [1, 37, 3000])
def test_merge_bit_exact(n):
    import torch
    import paper_1907_02814_amd as cmc
    rng = np.random.default_rng(100 + n)
    cap_d = rng.integers(0, 80, n)
    cap_s = rng.integers(0, 70, n)
    dst = _host_sp(rng, cap_d, np.minimum(rng.integers(-2, 90, n), cap_d + 3))
    src = _host_sp(rng, cap_s, rng.integers(-1, 80, n))
    cap_s[::7] = 200                      # cells with many products
    src = _host_sp(rng, cap_s, np.minimum(cap_s, rng.integers(0, 220, n)))
    gd, gs = _dev(dst), _dev(src)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    dr = cmc.merge_species(gd, gs, status=st, dropped=True)
    torch.cuda.synchronize()
    rd = O.merge_species(dst, src)
    _eq(gd, dst, "dst")
    _eq(gs, src, "src")
    assert np.array_equal(dr.cpu().numpy(), rd)
    assert bool(int(st.item()) & cmc.ST_OVERFLOW) == bool(rd.any())


@pytest.mark.parametrize("n,head", [(1, 0), (500, 5), (40000, 3)])
def test_rebin_bit_exact(n, head):
    import paper_1907_02814_amd as cmc
    rng = np.random.default_rng(200 + n)
    cap = rng.integers(0, 30, n)
    sp = _host_sp(rng, cap, rng.integers(-1, 35, n))
    g = cmc.rebin(_dev(sp), head)
    r = O.rebin(sp, head)
    _eq(g, r, "rebin")
    full = dict(sp, count=None)
    g = cmc.rebin(_dev(full), head)
    _eq(g, O.rebin(full, head), "rebin of a full species")


@pytest.mark.parametrize("precision", [0, 1])
def test_chained_steps_with_products_recycled(precision):
    """Three steps of all three processes on uneven cells; between steps the
    new electrons join the electrons (which then radiate and make Trident
    pairs) and the new positrons a positron population; every array is
    compared with the oracle doing the same."""
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import Parity
    rng = np.random.default_rng(31)
    wl = W.cfg3(rng, n_cells=48, dt=4e-13, lo=4, hi=600)
    wl.electrons = O.rebin(wl.electrons, 48)
    n = wl.n_cells
    pos = _host_sp(rng, np.full(n, 96), np.zeros(n), parent=True)
    for k in ("px", "py", "pz", "w"):
        pos[k][:] = 0.0
    pos["parent"][:] = -1
    P = Parity(wl, precision=precision)
    gpos = _dev(pos)
    merged = 0
    for s in range(3):
        P.step(s)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        de = cmc.merge_species(P.g.electrons, P.g.new_el, status=st, dropped=True)
        dp = cmc.merge_species(gpos, P.g.new_po, status=st, dropped=True)
        torch.cuda.synchronize()
        merged += int(P.ref.new_el["count"].sum())
        re_ = O.merge_species(P.ref.electrons, P.ref.new_el)
        rp = O.merge_species(pos, P.ref.new_po)
        assert np.array_equal(de.cpu().numpy(), re_) and np.array_equal(dp.cpu().numpy(), rp)
        for g, r, what in ((P.g.electrons, P.ref.electrons, "electrons"), (gpos, pos, "positrons")):
            assert np.array_equal(g["count"].cpu().numpy(), r["count"]), (s, what)
            for k in ("px", "py", "pz", "w"):
                a, b = g[k].cpu().numpy(), r[k]
                err = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
                assert np.all((a == b) | (err <= P.rtol)), (s, what, k, float(err.max()))
        assert not P.g.new_el["count"].cpu().numpy().any()
    # pairs were made and their electrons took part in the later steps
    assert merged > 0
