"""cmc_collide_step against the oracle, step by step (parity rules in
gpu_parity.py): FP64 form at 1e-12, FP32 form at 1e-5, bit-exact events,
slots and parents except counted near-threshold flips."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_02814_amd import workloads as W

pytestmark = pytest.mark.gpu
MEC2 = 0.51099895


def _run(wl, steps, **kw):
    from gpu_parity import Parity
    P = Parity(wl, **kw)
    for s in range(steps):
        P.step(s)
    print(f"[parity] {wl.name}: {P.flips} near-threshold flip(s) in {steps} step(s); "
          f"max relative error per output: " + ", ".join(f"{k} {v:.1e}" for k, v in P.errors.items()))
    assert P.flips <= max(1, wl.n_cells // 50)
    return P


def test_cfg1_physical_dt_ten_steps():
    # Plain FP64 Bremsstrahlung, 64 cells x (256 e + 256 Cu), dt = 0.1 fs
    _run(W.cfg1(), 10)


def test_cfg1_amplified_dt():
    # same cells with dt x 1e4 so that most pairs are tested near P ~ 0.3
    P = _run(W.cfg1(dt=1e-12), 3)
    assert P.ref.photons["count"].sum() > 1000


@pytest.mark.parametrize("precision", [0, 1])
def test_bethe_heitler_cells(precision):
    wl = W.cfg2(np.random.default_rng(5), n_cells=48, per_cell=1024, dt=3e-13)
    P = _run(wl, 2, precision=precision)
    assert (wl.photons["count"].sum() - P.ref.photons["count"].sum()) > 100


def _cycled_photons(n_cells, seed):
    """cfg2 cells (1024 Au ions of one weight) holding fewer photons than
    ions: the photon species is cycled, K = 1 .. 3 pairs per photon and
    e = N_i mod N_photon photons once more."""
    wl = W.cfg2(np.random.default_rng(seed), n_cells=n_cells, per_cell=1024, dt=3e-13)
    live = np.random.default_rng(seed + 1).integers(300, 1024, n_cells)
    live[:4] = (1023, 1000, 512, 341)        # e = 1, e = 24, K = 2 with e = 0, K = 3 with e = 1
    wl.photons["count"][:] = live
    return wl


@pytest.mark.parametrize("precision", [0, 1])
def test_cycled_photons_against_the_oracle(precision):
    wl = _cycled_photons(48, 41)
    P = _run(wl, 2, precision=precision)
    assert (wl.photons["count"].sum() - P.ref.photons["count"].sum()) > 50


@pytest.mark.parametrize("precision", [0, 1])
def test_few_mobile_particles_against_many_ions(precision):
    """One to seven electrons and photons per cell against 11000-12000 ions
    at rest of one weight: each mobile particle pairs K = N_i div N_m times
    (up to 12000; the repetition of an open pair needs 15 bits) and the e of
    smallest key once more, all three processes, amplified dt."""
    rng = np.random.default_rng(61)
    n = 24
    ne = rng.integers(1, 8, n)
    ng = rng.integers(1, 8, n)
    ni = rng.integers(11000, 12001, n)
    e_g = 1 + np.exp(rng.uniform(math.log(1.0), math.log(500.0), ne.sum())) / MEC2
    k = (1.022 + rng.exponential(5.0, ng.sum())) / MEC2
    Wi = np.repeat(5.9e28 / ni, ni)
    wl = W.assemble("few-mobile", 79, 3e-14, 7, 1, rng.uniform(0, 79, n), np.full(n, 5.9e28),
                    np.exp(rng.uniform(math.log(10), math.log(1e4), n)), e_g, np.repeat(5.9e28 / ni, ne), ne,
                    k, np.repeat(5.9e28 / ni, ng) * rng.lognormal(0, 1, ng.sum()), ng, Wi, ni, rng,
                    photon_extra=np.full(n, 64), pair_cap=np.full(n, 64))
    P = _run(wl, 2, precision=precision)
    I = P.state.ti.cpu().numpy().sum(0)
    assert I[0] == int(ni.sum()) and I[1] == int(ni.sum())   # N = N_ion pairs per cell and process
    assert I[3] + I[4] + I[5] > 5


@pytest.mark.parametrize("precision", [0, 1])
def test_events_on_cycled_particles_in_pair_order(precision):
    """A few electrons and photons per cell, each paired hundreds of times
    with the ions (one weight, at rest), at a time step that gives about
    every second electron an event in a step: an electron's later pairs see
    it as its earlier events left it, a converted photon pairs no more, and
    the products keep pair order (Sec. III.A), whichever kernel settles
    them."""
    rng = np.random.default_rng(83)
    n = 40
    ne = rng.integers(6, 15, n)
    ng = rng.integers(3, 10, n)
    ni = rng.integers(2500, 4001, n)
    e_g = 1 + np.exp(rng.uniform(math.log(5.0), math.log(500.0), ne.sum())) / MEC2
    k = (1.022 + rng.exponential(20.0, ng.sum())) / MEC2
    wl = W.assemble("cycled-events", 79, 3e-13, 7, 1, rng.uniform(0, 79, n), np.full(n, 5.9e28),
                    np.exp(rng.uniform(math.log(10), math.log(1e4), n)), e_g, np.repeat(5.9e28 / ni, ne), ne,
                    k, np.repeat(5.9e28 / ni, ng) * rng.lognormal(0, 1, ng.sum()), ng,
                    np.repeat(5.9e28 / ni, ni), ni, rng, photon_extra=np.full(n, 128), pair_cap=np.full(n, 128))
    P = _run(wl, 2, precision=precision)
    I = P.state.ti.cpu().numpy().sum(0)
    # the last step: an event for about every second electron (up to 20 in
    # a cell), and converted photons whose remaining pairs were not tested
    assert I[3] > int(ne.sum()) // 2
    assert I[5] > 0 and I[2] < I[0]


@pytest.mark.parametrize("precision", [0, 1])
def test_cycled_species_above_4096(precision):
    """Electrons and photons cycled against more ions, with more than 4096
    of them per cell (the bucket histogram of the sort holds 4096 entries):
    the per-particle bounds of both electron-ion processes and the ranks
    must not share it (Sec. III.A pairing, all three processes)."""
    rng = np.random.default_rng(71)
    n = 16
    ne = rng.integers(4100, 6000, n)
    ng = rng.integers(4100, 6000, n)
    ni = np.maximum(ne, ng) + rng.integers(1, 2000, n)
    e_g = 1 + np.exp(rng.uniform(math.log(1.0), math.log(500.0), ne.sum())) / MEC2
    k = (1.022 + rng.exponential(5.0, ng.sum())) / MEC2
    # a time step that leaves most cells one or two events, so that they keep
    # the pass kernel's candidates instead of the sequential step
    wl = W.assemble("cycled-large", 79, 3e-16, 7, 1, rng.uniform(0, 79, n), np.full(n, 5.9e28),
                    np.exp(rng.uniform(math.log(10), math.log(1e4), n)), e_g, np.repeat(5.9e28 / ni, ne), ne,
                    k, np.repeat(5.9e28 / ni, ng) * rng.lognormal(0, 1, ng.sum()), ng,
                    np.repeat(5.9e28 / ni, ni), ni, rng, photon_extra=np.full(n, 256), pair_cap=np.full(n, 256))
    P = _run(wl, 2, precision=precision)
    I = P.state.ti.cpu().numpy().sum(0)
    assert I[3] > 10


@pytest.mark.parametrize("precision", [0, 1])
def test_all_processes_uneven_cells(precision):
    wl = W.cfg3(np.random.default_rng(9), n_cells=160, dt=2e-13, lo=1, hi=3000)
    P = _run(wl, 2, precision=precision)
    I = P.state.ti.cpu().numpy().sum(0)
    assert I[3] > 100 and I[5] > 10


@pytest.mark.parametrize("precision", [0, 1])
def test_moving_ions_all_processes(precision):
    # Sec. III.A frame change: every pair is tested, sampled and given its
    # products in its ion's rest frame (ion proper velocities up to 0.5)
    wl = W.cfg3(np.random.default_rng(11), n_cells=96, dt=2e-13, lo=1, hi=2000)
    W.moving_ions(wl, np.random.default_rng(12), 0.5)
    P = _run(wl, 2, precision=precision)
    I = P.state.ti.cpu().numpy().sum(0)
    assert I[3] > 100 and I[4] > 0 and I[5] > 10


def test_moving_ions_bremsstrahlung_fp64():
    wl = W.moving_ions(W.cfg1(dt=1e-12), np.random.default_rng(13), 0.8)
    P = _run(wl, 2)
    assert P.ref.photons["count"].sum() > 1000


def _unequal_ion_weights(wl, rng):
    """Every other cell gets ions of unequal weight (log-normal factors):
    there the ion order enters n_ab and W_i/max(W, W_i)."""
    odd = np.repeat(np.arange(wl.n_cells) % 2 == 1, np.diff(wl.ions["off"]))
    wl.ions["w"][odd] *= rng.lognormal(0.0, 1.0, int(odd.sum()))
    return wl


@pytest.mark.parametrize("precision", [0, 1])
def test_unequal_ion_weights(precision):
    wl = _unequal_ion_weights(W.cfg3(np.random.default_rng(31), n_cells=96, dt=2e-13, lo=1, hi=2000),
                              np.random.default_rng(32))
    P = _run(wl, 2, precision=precision)
    I = P.state.ti.cpu().numpy().sum(0)
    assert I[3] > 100 and I[5] > 10


def test_foil_chain_cells():
    # foil cells with all three processes (the benchmark chain is Bremsstrahlung -> Bethe-Heitler)
    wl = W.cfg5(np.random.default_rng(2), n_cells=6, per_cell=4096, dt=5e-14, processes=7)
    P = _run(wl, 3)
    assert P.ref.photons["count"].sum() > 0


def _stream_cells(rng, bad=False):
    """Cells for the stream kernel (ions at rest, N_e >= N_i, 1024 < N_e <=
    4096) beside cells it leaves to the pass kernel: ions of unequal weight
    (cell 6), N_e above 4096 (cell 4), N_e = 1024 (the direct form, cell 5)
    and electrons cycled against more ions (cell 7).  bad: a NaN electron
    weight in cell 1 and a negative ion weight in cell 3."""
    ne = np.array([1025, 4096, 2000, 3000, 4097, 1024, 2500, 1500])
    ni = np.array([1025, 4096, 1, 2999, 4000, 1024, 2500, 1600])
    ng = np.array([0, 12, 3, 0, 5, 2, 40, 7])
    n = len(ne)
    n_i = np.full(n, 5.9e28)
    e_g = 1 + np.exp(rng.uniform(math.log(1.0), math.log(500.0), ne.sum())) / MEC2
    k = 2.0 + rng.exponential(5.0 / MEC2, ng.sum())
    iw = np.repeat(n_i / ni, ni)
    ioff = np.concatenate([[0], np.cumsum(ni)])
    iw[ioff[6]:ioff[7]] *= rng.lognormal(0.0, 1.0, ni[6])
    ew = np.repeat(n_i / ni, ne) * rng.lognormal(0.0, 1.0, ne.sum())
    if bad:
        ew[ne[0] + 17] = np.nan
        iw[ioff[3] + 5] = -1.0
    wl = W.assemble("stream-cells", 79, 2e-15, 7, 1, rng.uniform(0.0, 79.0, n), n_i, np.full(n, 100.0),
                    e_g, ew, ne, k, np.repeat(n_i / ni, ng) * rng.lognormal(0, 1, ng.sum()), ng, iw, ni, rng,
                    photon_extra=np.full(n, 512), pair_cap=np.full(n, 128))
    return wl


@pytest.mark.parametrize("precision", [0, 1])
def test_stream_kernel_cells(precision):
    """The electron-ion pass of the stream kernel and of the pass kernel's
    forms on the cells beside it, against the oracle (all processes)."""
    P = _run(_stream_cells(np.random.default_rng(51)), 3, precision=precision)
    I = P.state.ti.cpu().numpy()
    assert I[:, 3].sum() > 100


@pytest.mark.parametrize("precision", [0, 1])
def test_stream_kernel_filter_edges(precision):
    """Bremsstrahlung and Bethe-Heitler (no Trident), both forms: in the FP64
    form the stream kernel filters its bound tests in FP32 and tests the
    pairs that pass from their FP64 sigma v; the cells it lists go to the
    lane event kernel.  FP64: half the electrons sit 1e-9 to 1e-6
    (relative) from the emission threshold, the segment joins gamma = 2
    and 100 and the top of the tables, where FP32 energies may fall on the
    other side, or above the top (the status bit of energies above the
    tables).  None sits on a boundary itself: there the last bit of the
    FP64 energy (how its sum of squares is rounded) decides.  FP32: the
    form itself looks up FP32 energies, which this close to a join take
    the other segment's cross section, so only the electrons above the top
    are added.  The run must match the oracle."""
    import paper_1907_02814_amd as cmc
    rng = np.random.default_rng(83)
    ne = np.array([1100, 1500, 2048, 2500, 1200, 1800])
    ni = np.array([1100, 1400, 2048, 2000, 1200, 1700])
    ng = np.array([0, 9, 3, 0, 40, 5])
    n = len(ne)
    n_i = np.full(n, 5.9e28)
    tmin = 1e-3 / MEC2
    eps = np.array([-1e-6, -3e-8, -1e-9, 1e-9, 3e-8, 1e-6])
    edges = np.concatenate([2.0 * (1 + eps), 100.0 * (1 + eps), 1 + tmin * (1 + eps), 2e4 * (1 + eps), [3e4]])
    if precision == cmc.FP32:
        edges = np.array([3e4])
    e_g = 1 + np.exp(rng.uniform(math.log(1e-3), math.log(500.0), ne.sum())) / MEC2
    pick = rng.random(ne.sum()) < 0.5
    e_g[pick] = rng.choice(edges, int(pick.sum()))
    k = 2.0 + rng.exponential(5.0 / MEC2, ng.sum())
    wl = W.assemble("stream-edges", 79, 1.5e-15, int(cmc.BREMS | cmc.BH), 1, rng.uniform(0.0, 79.0, n), n_i,
                    np.full(n, 100.0), e_g, np.repeat(n_i / ni, ne) * rng.lognormal(0.0, 1.0, ne.sum()), ne, k,
                    np.repeat(n_i / ni, ng) * rng.lognormal(0, 1, ng.sum()), ng, np.repeat(n_i / ni, ni), ni, rng,
                    photon_extra=np.full(n, 512), pair_cap=np.full(n, 128))
    P = _run(wl, 3, precision=precision, schedule=cmc.SCHED_GROUP)
    I = P.state.ti.cpu().numpy()
    assert I[:, 3].sum() > 20
    assert int(P.state.status.item()) & cmc.ST_GAMMA_HIGH


@pytest.mark.parametrize("precision", [0, 1])
def test_lane_event_kernel_against_the_oracle(precision):
    """Foil cells, Bremsstrahlung and Bethe-Heitler, at a dt that opens zero
    to about ten pairs per cell: the cells the stream kernel lists go to the
    lane event kernel (up to eight open pairs) or the wavefront one."""
    import paper_1907_02814_amd as cmc
    wl = W.cfg5(np.random.default_rng(71), n_cells=32, per_cell=4096, dt=1.5e-16, processes=3)
    P = _run(wl, 3, precision=precision, schedule=cmc.SCHED_GROUP)
    assert P.state.ti.cpu().numpy()[:, 3].sum() > 20


def _bh_lane_cells(dt=5e-14, seed=91):
    """Cells for the lane event kernel with photon-ion pairs open: electrons
    below the emission threshold but for 0.2% of 0.1-1 MeV, photons of
    20-200 MeV cycled against the ions (10-256 of them), Bremsstrahlung and
    Bethe-Heitler.  At dt = 5e-14 s a few pairs open per cell; some cells
    convert a photon (handed on by the lane kernel), others do not."""
    import paper_1907_02814_amd as cmc
    rng = np.random.default_rng(seed)
    ne = np.array([1100, 1500, 2048, 1300, 1200, 1800, 1400, 1600])
    ni = ne.copy()
    ng = np.array([50, 120, 200, 256, 30, 90, 160, 10])
    n = len(ne)
    n_i = np.full(n, 5.9e28)
    e_g = 1 + rng.uniform(0.1e-3, 0.9e-3, ne.sum()) / MEC2
    hot = rng.random(ne.sum()) < 0.002
    e_g[hot] = 1 + rng.uniform(0.1, 1.0, int(hot.sum())) / MEC2
    k = np.exp(rng.uniform(math.log(20.0), math.log(200.0), ng.sum())) / MEC2
    return W.assemble("bh-lane", 79, dt, int(cmc.BREMS | cmc.BH), 1, rng.uniform(1.0, 79.0, n), n_i,
                      np.full(n, 100.0), e_g, np.repeat(n_i / ni, ne), ne, k,
                      np.repeat(n_i / ni, ng) * rng.lognormal(0, 1, ng.sum()), ng, np.repeat(n_i / ni, ni), ni, rng,
                      photon_extra=np.full(n, 64), pair_cap=np.full(n, 64))


@pytest.mark.parametrize("precision", [0, 1])
def test_lane_event_kernel_photon_pairs(precision):
    """The lane event kernel with photon-ion pairs among a cell's open
    pairs: cells without a conversion are applied by the lane, a conversion
    hands the cell on to the wavefront and workgroup kernels.  Against the
    oracle over three steps."""
    import paper_1907_02814_amd as cmc
    P = _run(_bh_lane_cells(), 3, precision=precision, schedule=cmc.SCHED_GROUP)
    I = P.state.ti.cpu().numpy()    # the last step's tallies
    assert I[:, 5].sum() > 0 and I[:, 3].sum() > 0


@pytest.mark.parametrize("schedule", ["GROUP", "SPLIT", "QUEUE"])
def test_stream_kernel_bad_weights(schedule):
    import paper_1907_02814_amd as cmc
    P = _run(_stream_cells(np.random.default_rng(52), bad=True), 2, precision=cmc.FP32,
             schedule=getattr(cmc, "SCHED_" + schedule))
    assert int(P.state.status.item()) & cmc.ST_BAD_WEIGHT
    I = P.state.ti.cpu().numpy()
    assert I[1, 0] == 0 and I[3, 0] == 0 and I[0, 0] > 0


def test_edge_cells():
    rng = np.random.default_rng(4)
    ne = np.array([0, 3, 1, 50, 7, 1, 200, 5])
    ng = np.array([4, 0, 1, 30, 7, 9, 0, 5])
    ni = np.array([6, 5, 1, 0, 7, 1, 17, 300])
    Zs = np.array([0.0, 29.0, 12.0, 3.0, 29.0, 0.0, 7.5, 1e-6])
    n = len(ne)
    e_g = 1 + np.exp(rng.uniform(math.log(0.002), math.log(1e4), ne.sum())) / MEC2
    k = 2.0 + np.exp(rng.uniform(math.log(1e-7), math.log(1e4), ng.sum()))
    wl = W.assemble("edges", 29, 1e-12, 7, 1, Zs, np.full(n, 8.5e28), np.array([1, 1e4, 50, 100, 3, 1, 1e3, 10.0]),
                    e_g, rng.lognormal(0, 1, ne.sum()) * 1e26, ne, k, rng.lognormal(0, 1, ng.sum()) * 1e26, ng,
                    rng.lognormal(0, 1, ni.sum()) * 1e26, ni, rng,
                    photon_extra=np.full(n, 2) , pair_cap=np.full(n, 3))
    _run(wl, 3)


def test_flags_bad_cells_and_limits():
    import paper_1907_02814_amd as cmc
    wl = W.cfg1(np.random.default_rng(1), n_cells=6, per_cell=32, dt=1e-12)
    wl.cells["Zstar"][1] = 30.0
    wl.cells["T_e"][2] = -1.0
    wl.ions["w"][3 * 32 + 4] = np.nan
    P = _run(wl, 1, max_per_cell=32)
    st = int(P.state.status.item())
    assert st & cmc.ST_BAD_CELL and st & cmc.ST_BAD_WEIGHT
    # a cell larger than max_per_cell is skipped and flagged
    wl2 = W.cfg1(np.random.default_rng(1), n_cells=3, per_cell=40, dt=1e-12)
    from gpu_parity import Parity
    Q = Parity(wl2, max_per_cell=39)
    Q.state.status.zero_()
    Q.state.step(0)
    import torch
    torch.cuda.synchronize()
    assert int(Q.state.status.item()) & cmc.ST_TOO_LARGE
    assert Q.state.ti.cpu().numpy().sum() == 0


def test_overflow_drops_in_pair_order():
    wl = W.cfg1(np.random.default_rng(8), n_cells=8, per_cell=64, dt=3e-12)
    wl.photons = W._slab(np.full(8, 5))
    P = _run(wl, 1)
    assert P.state.ti.cpu().numpy()[:, 9].sum() > 0


def test_repeatable_bitwise():
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    wl = W.cfg3(np.random.default_rng(3), n_cells=64, dt=2e-13, lo=1, hi=2000)
    outs = []
    for _ in range(2):
        g = wl.copy().to_torch("cuda:0")
        st = cmc.StepState(gpu_tables(wl.Z), g.cells, g.electrons, g.photons, g.ions, g.new_el,
                           g.new_po, dt=wl.dt, seed=3, processes=wl.processes)
        for s in range(2):
            st.step(s)
        torch.cuda.synchronize()
        outs.append([g.electrons["px"].cpu().numpy(), g.photons["px"].cpu().numpy(),
                     g.new_po["pz"].cpu().numpy(), st.td.cpu().numpy(), st.ti.cpu().numpy()])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
