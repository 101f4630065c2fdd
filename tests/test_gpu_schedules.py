"""Schedules and graph replay of cmc_collide_step.

- Workgroup and wavefront teams, the hybrid of both, and workgroups taking
  the cells from the cost-sorted work queue give bit-identical results: the
  densities and n_ab are summed in one canonical order whatever the team
  shape, and every draw is keyed by where it is used.
- The sequential schedule (one workgroup per cell, pairs in order) gives the
  same events, counts and live slots; floating-point values agree to rounding
  (another kernel may contract a * b + c into a fused multiply-add
  differently, and sums the tallies in another order).
- A step captured in a HIP graph with the step number in device memory
  replays step after step exactly like eager steps.
"""
import numpy as np
import pytest

from paper_1907_02814_amd import workloads as W

pytestmark = pytest.mark.gpu

ARRAYS = [("electrons", k) for k in ("px", "py", "pz")] + \
         [(sp, k) for sp in ("photons", "new_el", "new_po") for k in ("px", "py", "pz", "w", "count")]


def _state(wl, schedule, precision):
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    g = wl.copy().to_torch("cuda:0")
    st = cmc.StepState(gpu_tables(wl.Z), g.cells, g.electrons, g.photons, g.ions, g.new_el, g.new_po,
                       dt=wl.dt, seed=7, processes=wl.processes, precision=precision, schedule=schedule)
    return g, st


def _live(g, out):
    """Slots past a cell's live count hold no particle: zeroed before a
    comparison (the schedules may leave different values there)."""
    for sp in ("photons", "new_el", "new_po"):
        off = getattr(g, sp)["off"].cpu().numpy()
        cnt = out[f"{sp}.count"]
        idx = np.arange(off[-1])
        cell = np.searchsorted(off, idx, side="right") - 1
        dead = idx - off[cell] >= cnt[cell]
        for k in ("px", "py", "pz", "w"):
            out[f"{sp}.{k}"][dead] = 0.0
    return out


def _snap(g, st):
    import torch
    torch.cuda.synchronize()
    out = {f"{sp}.{k}": getattr(g, sp)[k].cpu().numpy().copy() for sp, k in ARRAYS}
    out["ti"] = st.ti.cpu().numpy().copy()
    out["td"] = st.td.cpu().numpy().copy()
    out["status"] = int(st.status.item())
    return out


def _sched(name):
    """SCHED_<name>; a trailing "-" adds CMC_SCHED_NO_STREAM (no stream kernel)"""
    import paper_1907_02814_amd as cmc
    if name.endswith("-"):
        return getattr(cmc, "SCHED_" + name[:-1]) | cmc.SCHED_NO_STREAM
    return getattr(cmc, "SCHED_" + name)


@pytest.mark.parametrize("precision,other,hi,moving", [(0, "WAVE", 480, False), (1, "WAVE", 480, False),
                                                       (0, "GROUP-", 3000, False), (1, "GROUP-", 3000, "weights"),
                                                       (1, "QUEUE-", 3000, False),
                                                       (1, "HYBRID", 3000, False), (0, "HYBRID", 3000, True),
                                                       (1, "WAVE", 480, "weights"), (0, "QUEUE", 3000, False),
                                                       (1, "QUEUE", 3000, "weights"), (1, "QUEUE", 3000, True),
                                                       (0, "SPLIT", 3000, False), (1, "SPLIT", 3000, "weights"),
                                                       (1, "SPLIT", 3000, True)])
def test_team_shapes_bit_identical(precision, other, hi, moving):
    import paper_1907_02814_amd as cmc
    wl = W.cfg3(np.random.default_rng(21), n_cells=128, dt=2e-13, lo=1, hi=hi)
    if moving == "weights":       # ions of unequal weight in every other cell
        odd = np.repeat(np.arange(wl.n_cells) % 2 == 1, np.diff(wl.ions["off"]))
        wl.ions["w"][odd] *= np.random.default_rng(25).lognormal(0.0, 1.0, int(odd.sum()))
    elif moving:
        W.moving_ions(wl, np.random.default_rng(23), 0.5)
    ga, sa = _state(wl, cmc.SCHED_GROUP, precision)
    gb, sb = _state(wl, _sched(other), precision)
    for s in range(3):
        sa.step(s)
        sb.step(s)
        A, B = _snap(ga, sa), _snap(gb, sb)
        for k in A:
            assert np.array_equal(A[k], B[k]), (s, k)
    assert A["ti"][:, 3:6].sum() > 50


@pytest.mark.parametrize("precision,moving", [(0, False), (1, False), (1, True)])
def test_sequential_schedule_agrees(precision, moving):
    import paper_1907_02814_amd as cmc
    wl = W.cfg3(np.random.default_rng(22), n_cells=128, dt=2e-13, lo=1, hi=1500)
    if moving:
        W.moving_ions(wl, np.random.default_rng(24), 0.5)
    ga, sa = _state(wl, cmc.SCHED_AUTO, precision)
    gb, sb = _state(wl, cmc.SCHED_CELL, precision)
    for s in range(3):
        sa.step(s)
        sb.step(s)
        A, B = _live(ga, _snap(ga, sa)), _live(gb, _snap(gb, sb))
        for k in A:
            if k == "status" or k == "ti" or k.endswith("count"):
                assert np.array_equal(A[k], B[k]), (s, k)
            else:
                sc = np.maximum(np.abs(B[k]), 1e-300)
                err = np.max(np.abs(A[k] - B[k]) / sc) if np.size(B[k]) else 0.0
                assert err <= (1e-12 if precision == 0 else 1e-6), (s, k, err)
    assert A["ti"][:, 3:6].sum() > 50


@pytest.mark.parametrize("schedule", ["AUTO", "QUEUE", "SPLIT", "QUEUE-"])
def test_graph_replay_matches_eager_steps(schedule):
    """(the work queue is rebuilt and drained inside the captured step)"""
    import torch
    import paper_1907_02814_amd as cmc
    wl = W.cfg3(np.random.default_rng(23), n_cells=96, dt=2e-13, lo=1, hi=1200)
    sched = _sched(schedule)
    ge, se = _state(wl, sched, cmc.FP32)
    gg, sg = _state(wl, sched, cmc.FP32)
    se.step(0)
    sg.step(0)
    graph, counter = sg.graph(1)
    for s in range(1, 5):
        se.step(s)
        graph.replay()
        # eager work of the program between replays
        x = torch.arange(4096, device="cuda:0", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        assert float(x.item()) == 4096 * 4095 / 2
        A, B = _snap(ge, se), _snap(gg, sg)
        for k in A:
            assert np.array_equal(A[k], B[k]), (s, k)
        assert int(counter.item()) == s + 1
    assert A["ti"][:, 3:6].sum() > 20


@pytest.mark.parametrize("precision,other", [(0, "WAVE"), (1, "WAVE"), (1, "HYBRID"), (1, "SPLIT")])
def test_cycled_photons_bit_identical_across_team_shapes(precision, other):
    """Cells with fewer photons than ions (300-1023 photons, 1024 ions of one
    weight): workgroup teams take the direct form with the selection of the
    photons that pair once more, wavefront teams (at most 256 pairs in their
    direct form) the ordered form; both give the same bits."""
    import paper_1907_02814_amd as cmc
    from test_gpu_step import _cycled_photons
    wl = _cycled_photons(64, 43)
    ga, sa = _state(wl, cmc.SCHED_GROUP, precision)
    gb, sb = _state(wl, getattr(cmc, "SCHED_" + other), precision)
    for s in range(3):
        sa.step(s)
        sb.step(s)
        A, B = _snap(ga, sa), _snap(gb, sb)
        for k in A:
            assert np.array_equal(A[k], B[k]), (s, k)
    assert A["ti"][:, 5].sum() > 20


@pytest.mark.parametrize("precision,processes", [(0, 7), (1, 7), (0, 3), (1, 3)])
def test_foil_cells_bit_identical_across_schedules(precision, processes):
    """Foil cells (4096 electrons + 4096 Au ions, the photons of earlier steps
    cycled against the ions): the stream kernel with workgroup teams, with
    wavefront teams (SPLIT) and from the work queue, and the same schedules
    without it, give the same bits.  Without Trident (processes 3) the cells
    the stream kernel lists go to the lane event kernel, the others' to the
    wavefront one."""
    import paper_1907_02814_amd as cmc
    wl = W.cfg5(np.random.default_rng(61), n_cells=48, per_cell=4096, dt=4e-15, processes=processes)
    states = [_state(wl, _sched(s), precision) for s in ("GROUP", "SPLIT", "QUEUE", "GROUP-", "QUEUE-", "SPLIT-")]
    for s in range(4):
        snaps = []
        for g, st in states:
            st.step(s)
            snaps.append(_snap(g, st))
        for other in snaps[1:]:
            for k in snaps[0]:
                assert np.array_equal(snaps[0][k], other[k]), (s, k)
    assert snaps[0]["ti"][:, 3].sum() > 1000 and snaps[0]["ti"][:, 2].sum() > 0


@pytest.mark.parametrize("precision", [0, 1])
def test_lane_event_kernel_bit_identical(precision):
    """Foil cells (Bremsstrahlung and Bethe-Heitler) at a dt that opens zero
    to about ten pairs per cell: the lane event kernel, which takes the cells
    the stream kernel lists with up to eight open pairs, and the wavefront
    event kernel (the same schedule without the stream kernel) give the same
    bits over four steps."""
    wl = W.cfg5(np.random.default_rng(67), n_cells=64, per_cell=4096, dt=1.5e-16, processes=3)
    states = [_state(wl, _sched(s), precision) for s in ("GROUP", "GROUP-", "SPLIT")]
    events = 0
    for s in range(4):
        snaps = []
        for g, st in states:
            st.step(s)
            snaps.append(_snap(g, st))
        for other in snaps[1:]:
            for k in snaps[0]:
                assert np.array_equal(snaps[0][k], other[k]), (s, k)
        events += int(snaps[0]["ti"][:, 3].sum())
    assert events > 100


@pytest.mark.parametrize("precision", [0, 1])
def test_lane_event_kernel_photon_pairs_bit_identical(precision):
    """Cells with photon-ion pairs open (some converting): the lane event
    kernel after the stream kernel, and the wavefront and workgroup event
    kernels without it, give the same bits over four steps."""
    from test_gpu_step import _bh_lane_cells
    wl = _bh_lane_cells()
    states = [_state(wl, _sched(s), precision) for s in ("GROUP", "GROUP-", "SPLIT")]
    for s in range(4):
        snaps = []
        for g, st in states:
            st.step(s)
            snaps.append(_snap(g, st))
        for other in snaps[1:]:
            for k in snaps[0]:
                assert np.array_equal(snaps[0][k], other[k]), (s, k)
