"""Parity at the benchmark sizes, in the launch configuration bench.py times
(automatic schedule): cfg2 in full (4096 cells x (1024 photons + 1024 Au
ions), both forms) against the oracle; foil-chain cells at their full size
(4096 electrons + 4096 Au ions, all processes); cfg5 in full and cfg3 in
full (16384 uneven cells, all processes), both forms over three steps, on
the GPU against the oracle on a sample of their cells (the random numbers
are keyed by the global cell index); the expected yield and its adjoint on
cfg4 in full (1024 cells x 4096 electrons), both forms, against the oracle
on every cell and electron."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_02814_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_cfg2_full_size_fp32():
    import paper_1907_02814_amd as cmc
    from gpu_parity import Parity
    wl = W.cfg2()
    P = Parity(wl, precision=cmc.FP32)
    for s in range(2):
        P.step(s)
    print(f"[parity] cfg2 full: {P.flips} flip(s); " + ", ".join(f"{k} {v:.1e}" for k, v in P.errors.items()))
    assert P.flips <= 2
    assert P.state.ti.cpu().numpy()[:, 2].sum() > 4_000_000


def test_foil_cells_full_size_fp32():
    import paper_1907_02814_amd as cmc
    from gpu_parity import Parity
    wl = W.cfg5(np.random.default_rng(1005), n_cells=192)
    P = Parity(wl, precision=cmc.FP32)
    for s in range(2):
        P.step(s)
    print(f"[parity] cfg5 cells: {P.flips} flip(s); " + ", ".join(f"{k} {v:.1e}" for k, v in P.errors.items()))
    assert P.flips <= 2
    assert P.ref.photons["count"].sum() > 0


@pytest.mark.parametrize("precision", [1, 0])
def test_cfg5_full_size_sampled_cells(precision):
    """cfg5 in full (131072 cells x (4096 electrons + 4096 Au ions),
    generated in HBM, about 125 GB), in the launch configuration bench.py
    times, three steps of the Bremsstrahlung -> Bethe-Heitler chain: 1024
    seeded cells (the bench's oracle sample) against the oracle run on the
    same cells with their global ids, after every step."""
    import gc
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import compare_host_subsets, gpu_tables
    g = W.cfg5_device("cuda:0")
    n = g.cells["Zstar"].numel()
    assert n == 131072 and int(g.electrons["off"][-1].item()) == 131072 * 4096
    sample = np.sort(np.random.default_rng(1005).choice(n, 1024, replace=False))
    ref = g.host_subset(sample)
    st = cmc.StepState(gpu_tables(79), g.cells, g.electrons, g.photons, g.ions, g.new_el, g.new_po, dt=g.dt,
                       seed=1, processes=g.processes, precision=precision)
    rtol = 1e-12 if precision == cmc.FP64 else 1e-5
    skip = np.zeros(len(sample), bool)
    events = 0
    try:
        for s in range(3):
            st.step(s)
            torch.cuda.synchronize()
            oti, otd, ost = O.collide_step(O.tables(79), ref.cells, ref.electrons, ref.photons, ref.ions,
                                           ref.new_el, ref.new_po, g.dt, 1, s, g.processes)
            ti = st.ti.cpu().numpy()[sample]
            td = st.td.cpu().numpy()[sample]
            now = g.host_subset(sample)
            skip, errs = compare_host_subsets(ti, td, now, ref, oti, otd, rtol, skip)
            events += int(oti[:, 3:6].sum())
            print(f"[parity] cfg5 full, precision {precision}, step {s}: {int(skip.sum())} cell(s) left out "
                  f"(near threshold); " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
        assert int(st.status.item()) == 0
        assert skip.sum() <= 4
        assert events > 500
    finally:
        del st, g
        gc.collect()
        torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [1, 0])
def test_cfg3_full_sampled_cells(precision):
    """cfg3 in full (16384 uneven cells, all processes), in the batched
    schedule the benchmark uses for it (automatic: the work queue), three
    steps: 256 seeded cells and the 8 largest against the oracle run on the
    same cells with their global ids, after every step."""
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import compare_host_subsets, gpu_tables
    wl = W.cfg3()
    g = wl.copy().to_torch("cuda:0")
    st = cmc.StepState(gpu_tables(wl.Z), g.cells, g.electrons, g.photons, g.ions, g.new_el, g.new_po,
                       dt=wl.dt, seed=1, processes=wl.processes, precision=precision)
    sample = np.sort(np.random.default_rng(5).choice(wl.n_cells, 256, replace=False))
    big = np.argsort(np.diff(wl.electrons["off"]) + np.diff(wl.ions["off"]))[-8:]
    sample = np.unique(np.concatenate([sample, big]))
    ref = g.host_subset(sample)
    rtol = 1e-12 if precision == cmc.FP64 else 1e-5
    skip = np.zeros(len(sample), bool)
    pairs = 0
    for s in range(3):
        st.step(s)
        torch.cuda.synchronize()
        oti, otd, ost = O.collide_step(O.tables(wl.Z), ref.cells, ref.electrons, ref.photons, ref.ions,
                                       ref.new_el, ref.new_po, wl.dt, 1, s, wl.processes)
        now = g.host_subset(sample)
        skip, errs = compare_host_subsets(st.ti.cpu().numpy()[sample], st.td.cpu().numpy()[sample], now, ref,
                                          oti, otd, rtol, skip)
        pairs += int(oti[:, 0:3].sum())
        print(f"[parity] cfg3 full, precision {precision}, step {s}: {int(skip.sum())} cell(s) left out "
              f"(near threshold); " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    assert skip.sum() <= 4
    assert pairs > 3e5


def test_cfg2_full_size_fp64():
    import paper_1907_02814_amd as cmc
    from gpu_parity import Parity
    wl = W.cfg2()
    P = Parity(wl, precision=cmc.FP64)
    for s in range(2):
        P.step(s)
    print(f"[parity] cfg2 full FP64: {P.flips} flip(s); " + ", ".join(f"{k} {v:.1e}" for k, v in P.errors.items()))
    assert P.flips <= 2
    assert P.state.ti.cpu().numpy()[:, 2].sum() > 4_000_000


@pytest.mark.parametrize("precision,rtol", [(0, 1e-12), (1, 1e-5)])
def test_cfg4_expected_yield_full_size(precision, rtol):
    import torch
    import paper_1907_02814_amd as cmc
    from gpu_parity import gpu_tables
    from test_gpu_yield import check_adjoint
    y = W.cfg4()
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in y.items() if isinstance(v, np.ndarray)}
    args = (g["Zstar"], g["n_e"], g["T_e"], g["off"], g["px"], g["py"], g["pz"], g["w"], y["dt"])
    oargs = (y["Zstar"], y["n_e"], y["T_e"], y["off"], y["px"], y["py"], y["pz"], y["w"], y["dt"])
    Y = cmc.expected_yield(gpu_tables(29), *args, precision).cpu().numpy()
    Yo = O.expected_yield(O.tables(29), *oargs)
    print(f"[parity] cfg4 yield, precision {precision}: max rel {np.max(np.abs(Y - Yo) / np.abs(Yo)):.1e}")
    np.testing.assert_allclose(Y, Yo, rtol=rtol, atol=0)
    gY = np.linspace(0.5, 2.0, len(y["Zstar"]))
    G = cmc.expected_yield_backward(gpu_tables(29), *args, torch.from_numpy(gY).cuda(), precision)
    Go = O.expected_yield_backward(O.tables(29), *oargs, gY, scale=True)
    # every electron, knots included: both forms take the interval of the FP64 energy
    check_adjoint(G, Go, rtol, f"cfg4 full, precision {precision}")
